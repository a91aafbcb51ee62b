// One instantiation of the join kernels (see join_impl.h) for the row type
// VJ_JOIN_ELEM (float or uint8_t) and the padded row width VJ_JOIN_DP; the
// build compiles this file once per (type, width) so the instantiations
// compile in parallel.  Defines launch_join_<f32|u8>_<DP>.
#include "join_impl.h"

#if !defined(VJ_JOIN_ELEM) || !defined(VJ_JOIN_DP) || !defined(VJ_JOIN_FN)
#error "build with -DVJ_JOIN_ELEM=<float|uint8_t> -DVJ_JOIN_DP=<width> -DVJ_JOIN_FN=<name>"
#endif

namespace vj {
bool VJ_JOIN_FN(const JoinLaunch &L, hipStream_t s) { return wj::launch_dp<VJ_JOIN_ELEM, VJ_JOIN_DP>(L, s); }
}  // namespace vj
