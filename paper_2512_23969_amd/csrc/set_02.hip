// set_02.hip -- kernels and host launch code of parameter set 2 (SHA2-192f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(2)
