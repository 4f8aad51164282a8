// set_05.hip -- kernels and host launch code of parameter set 5 (SHA2-192s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(5)
