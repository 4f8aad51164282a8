// set_08_fused.hip -- the fused persistent kernel of parameter set 8 (SHAKE-192f)
// in every compiled shape (trees per FORS group, leaves per lane, waves per
// workgroup), its selector and its occupancy query.
#include "set_impl.hpp"

SLH_DEFINE_FUSED_SELECTOR(8)
