// set_09_fors.hip -- the FORS kernels of parameter set 9 (SHAKE-256f) in every
// compiled shape and instruction variant, and their selector.
#include "set_impl.hpp"

SLH_DEFINE_FORS_SELECTOR(9)
