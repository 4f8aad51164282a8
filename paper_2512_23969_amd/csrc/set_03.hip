// set_03.hip -- kernels and host launch code of parameter set 3 (SHA2-256f);
// its FORS, TREE and fused selectors compile in set_03_fors.hip,
// set_03_tree.hip and set_03_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(3)
SLH_DEFINE_SET_OPS(3)
