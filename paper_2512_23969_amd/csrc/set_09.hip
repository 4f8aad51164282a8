// set_09.hip -- kernels and host launch code of parameter set 9 (SHAKE-256f);
// its FORS, TREE and fused selectors compile in set_09_fors.hip,
// set_09_tree.hip and set_09_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(9)
SLH_DEFINE_SET_OPS(9)
