// set_09.hip -- kernels and host launch code of parameter set 9 (SHAKE-256f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(9)
