// set_03.hip -- kernels and host launch code of parameter set 3 (SHA2-256f);
// its FORS and TREE selectors compile in set_03_fors.hip and set_03_tree.hip.
#include "set_impl.hpp"

SLH_EXTERN_SELECTORS(3)
SLH_DEFINE_SET_OPS(3)
