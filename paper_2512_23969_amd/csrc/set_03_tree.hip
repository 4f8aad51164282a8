// set_03_tree.hip -- the TREE kernels of parameter set 3 (SHA2-256f) in every
// compiled block size, instruction variant and layer order, and their
// selector.
#include "set_impl.hpp"

SLH_DEFINE_TREE_SELECTOR(3)
