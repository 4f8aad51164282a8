// set_08.hip -- kernels and host launch code of parameter set 8 (SHAKE-192f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(8)
