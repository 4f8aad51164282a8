// set_03_fused.hip -- the fused persistent kernel of parameter set 3 (SHA2-256f)
// in every compiled shape (trees per FORS group, leaves per lane, waves per
// workgroup), its selector and its occupancy query.
#include "set_impl.hpp"

SLH_DEFINE_FUSED_SELECTOR(3)
