// set_06.hip -- kernels and host launch code of parameter set 6 (SHA2-256s).
#include "set_impl.hpp"

SLH_DEFINE_SET_OPS(6)
