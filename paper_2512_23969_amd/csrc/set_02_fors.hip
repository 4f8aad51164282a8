// set_02_fors.hip -- the FORS kernels of parameter set 2 (SHA2-192f) in every
// compiled shape and instruction variant, and their selector.
#include "set_impl.hpp"

SLH_DEFINE_FORS_SELECTOR(2)
