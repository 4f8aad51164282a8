// set_08_tree.hip -- the TREE kernels of parameter set 8 (SHAKE-192f) in every
// compiled block size, instruction variant and layer order, and their
// selector.
#include "set_impl.hpp"

SLH_DEFINE_TREE_SELECTOR(8)
