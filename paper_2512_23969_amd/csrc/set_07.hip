// set_07.hip -- kernels and host launch code of parameter set 7 (SHAKE-128f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(7)
