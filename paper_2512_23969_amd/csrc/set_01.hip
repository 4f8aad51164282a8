// set_01.hip -- kernels and host launch code of parameter set 1 (SHA2-128f);
// its FORS, TREE and fused selectors compile in set_01_fors.hip,
// set_01_tree.hip and set_01_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(1)
SLH_DEFINE_SET_OPS(1)
