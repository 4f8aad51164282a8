// set_08.hip -- kernels and host launch code of parameter set 8 (SHAKE-192f);
// its FORS, TREE and fused selectors compile in set_08_fors.hip,
// set_08_tree.hip and set_08_fused.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(8)
SLH_DEFINE_SET_OPS(8)
