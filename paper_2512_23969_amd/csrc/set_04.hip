// set_04.hip -- kernels and host launch code of parameter set 4 (SHA2-128s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(4)
