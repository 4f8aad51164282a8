// set_01.hip -- kernels and host launch code of parameter set 1 (SHA2-128f);
// its FORS and TREE selectors compile in set_01_fors.hip and set_01_tree.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(1)
SLH_DEFINE_SET_OPS(1)
