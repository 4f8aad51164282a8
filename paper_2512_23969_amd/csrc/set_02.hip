// set_02.hip -- kernels and host launch code of parameter set 2 (SHA2-192f);
// its FORS, TREE and fused selectors compile in set_02_fors.hip,
// set_02_tree.hip and set_02_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(2)
SLH_DEFINE_SET_OPS(2)
