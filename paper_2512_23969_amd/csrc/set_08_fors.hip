// set_08_fors.hip -- the FORS kernels of parameter set 8 (SHAKE-192f) in every
// compiled shape and instruction variant, and their selector.
#include "set_impl.hpp"

SLH_DEFINE_FORS_SELECTOR(8)
