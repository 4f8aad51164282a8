// set_07.hip -- kernels and host launch code of parameter set 7 (SHAKE-128f);
// its FORS and TREE selectors compile in set_07_fors.hip and set_07_tree.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(7)
SLH_DEFINE_SET_OPS(7)
