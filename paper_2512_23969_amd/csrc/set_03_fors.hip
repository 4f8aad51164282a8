// set_03_fors.hip -- the FORS kernels of parameter set 3 (SHA2-256f) in every
// compiled shape and instruction variant, and their selector.
#include "set_impl.hpp"

SLH_DEFINE_FORS_SELECTOR(3)
