// set_01.hip -- kernels and host launch code of parameter set 1 (SHA2-128f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(1)
