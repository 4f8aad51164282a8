// set_12.hip -- kernels and host launch code of parameter set 12 (SHAKE-256s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(12)
