// set_01_fused.hip -- the fused persistent kernel of parameter set 1 (SHA2-128f)
// in every compiled shape (trees per FORS group, leaves per lane, waves per
// workgroup), its selector and its occupancy query.
#include "set_impl.hpp"

SLH_DEFINE_FUSED_SELECTOR(1)
