// set_07_tree.hip -- the TREE kernels of parameter set 7 (SHAKE-128f) in every
// compiled block size, instruction variant and layer order, and their
// selector.
#include "set_impl.hpp"

SLH_DEFINE_TREE_SELECTOR(7)
