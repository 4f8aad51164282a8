// set_01_fors.hip -- the FORS kernels of parameter set 1 (SHA2-128f) in every
// compiled shape and instruction variant, and their selector.
#include "set_impl.hpp"

SLH_DEFINE_FORS_SELECTOR(1)
