// Join kernels over float rows (see join_impl.h).
#include "join_impl.h"

namespace vj {
bool launch_join_f32(const JoinLaunch &L, hipStream_t s) { return wj::launch_elem<float>(L, s); }
}  // namespace vj
