// Join kernels over uint8_t rows (see join_impl.h).
#include "join_impl.h"

namespace vj {
bool launch_join_u8(const JoinLaunch &L, hipStream_t s) { return wj::launch_elem<uint8_t>(L, s); }
}  // namespace vj
