// set_11.hip -- kernels and host launch code of parameter set 11 (SHAKE-192s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(11)
