// set_03.hip -- kernels and host launch code of parameter set 3 (SHA2-256f).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(3)
