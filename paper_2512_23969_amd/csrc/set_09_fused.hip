// set_09_fused.hip -- the fused persistent kernel of parameter set 9 (SHAKE-256f)
// in every compiled shape (trees per FORS group, leaves per lane, waves per
// workgroup), its selector and its occupancy query.
#include "set_impl.hpp"

SLH_DEFINE_FUSED_SELECTOR(9)
