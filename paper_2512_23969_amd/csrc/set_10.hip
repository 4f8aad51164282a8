// set_10.hip -- kernels and host launch code of parameter set 10 (SHAKE-128s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(10)
