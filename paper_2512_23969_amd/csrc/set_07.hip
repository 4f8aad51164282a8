// set_07.hip -- kernels and host launch code of parameter set 7 (SHAKE-128f);
// its FORS, TREE and fused selectors compile in set_07_fors.hip,
// set_07_tree.hip and set_07_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(7)
SLH_DEFINE_SET_OPS(7)
