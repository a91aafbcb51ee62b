// Row-width dispatch of the join kernels: one function per (row type,
// padded width), each compiled from join_inst.hip.
#include "vj_internal.h"

namespace vj {

#define VJ_WIDTHS(X) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define VJ_DECL(dp)                                               \
    bool launch_join_f32_##dp(const JoinLaunch &, hipStream_t);   \
    bool launch_join_u8_##dp(const JoinLaunch &, hipStream_t);    \
    bool launch_join_bf16_##dp(const JoinLaunch &, hipStream_t);  \
    bool launch_join_f8_##dp(const JoinLaunch &, hipStream_t);
VJ_WIDTHS(VJ_DECL)
#undef VJ_DECL

bool launch_join_f32(const JoinLaunch &L, hipStream_t s) {
    switch (L.dp) {
#define VJ_CASE(dp) case dp: return launch_join_f32_##dp(L, s);
        VJ_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: return false;
    }
}

bool launch_join_u8(const JoinLaunch &L, hipStream_t s) {
    switch (L.dp) {
#define VJ_CASE(dp) case dp: return launch_join_u8_##dp(L, s);
        VJ_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: return false;
    }
}

bool launch_join_bf16(const JoinLaunch &L, hipStream_t s) {
    switch (L.dp) {
#define VJ_CASE(dp) case dp: return launch_join_bf16_##dp(L, s);
        VJ_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: return false;
    }
}

bool launch_join_f8(const JoinLaunch &L, hipStream_t s) {
    switch (L.dp) {
#define VJ_CASE(dp) case dp: return launch_join_f8_##dp(L, s);
        VJ_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: return false;
    }
}

}  // namespace vj
