// Register-row MFMA sweeps (Kp <= 256): the rows' bf16 fragments stay in
// VGPRs while column tiles of 32 rows stream through a ring of LDS stages
// filled by direct global-to-LDS loads.  Shared by the kNN sweep of the
// graph build and the brute-force epsilon-join.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vj {
namespace ring {

// Shape of one (NSPLIT, KP) instantiation: RT row tiles of 16 per wave,
// tiles of BN columns staged KC dimensions at a time (KC = KP up to 256;
// wider rows in NCH chunks of 128 dimensions, else 192, else 64: small
// stages keep three or more of them in flight), staged rows of CPR + 1 chunks of 16 bytes (one pad chunk spreads a
// fragment read's 16 rows over distinct banks), IPW load instructions per
// wave and part per stage, each stage holding TERMS parts plus two 256-byte
// slots per wave (the tile's norms and ids), NB stages.
template <int NSPLIT, int KP>
struct Shape {
    static constexpr int KS = KP / 32;                 // MFMA k-steps of 32
    static constexpr int TERMS = NSPLIT == 3 ? 2 : 1;  // hi (+ lo) parts
    static constexpr int RT = TERMS * 16 * KS <= 64 ? 4 : KP <= 256 ? 2 : 1;
    static constexpr int CT = 2;
    static constexpr int BN = 16 * CT;                 // columns per tile
    static constexpr int ROWS = 4 * RT * 16;           // rows per workgroup
    static constexpr int KC = KP <= 256 ? KP
                              : KP % 128 == 0 ? 128
                              : KP % 192 == 0 ? 192 : 64;  // dimensions per stage
    static constexpr int NCH = KP / KC;                // stages per tile
    static constexpr int KCS = KC / 32;                // k-steps per stage
    static constexpr int CPR = KC / 8;                 // 16-byte chunks per staged row
    static constexpr int SPR = CPR + 1;                // staged slots per row
    static constexpr int IPW = (BN * SPR + 255) / 256; // load instructions per wave and part
    static constexpr int PART = 4 * IPW * 1024;        // bytes of one part of a stage
    // + each wave's copy of the tile's |x|^2 and node ids
    static constexpr int STAGE = TERMS * PART + 2 * 4 * 256;
    static constexpr int NB0 = (78 * 1024) / STAGE;  // two workgroups per CU fit in 160 KB
    static constexpr int NB = NB0 > 8 ? 8 : NB0;       // stages in the ring
    static constexpr int LPT = TERMS * IPW + 2;        // load instructions per wave and stage
    // the rows' fragments stay within 128 VGPRs
    static constexpr bool OK = KP % 32 == 0 && KP <= 1024 && TERMS * RT * KS * 4 <= 128 &&
                               NB >= 3 && (NB - 2) * LPT <= 60;
    // the kNN sweep stages whole rows
    static constexpr bool WHOLE = NCH == 1;
};

// one direct global-to-LDS load per lane: 16 bytes (or 4) from the
// wave-uniform base plus the lane's byte offset, to LDS byte address
// lds + 16 * lane (4 * lane); lds must be wave-uniform.  M0 is saved and
// restored inside the block.
__device__ __forceinline__ void lds_dma16(const void *base, uint32_t off, uint32_t lds) {
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
                 "global_load_lds_dwordx4 %2, %3\n\ts_nop 0\n\ts_mov_b32 m0, %0"
                 : "=&s"(saved) : "s"(lds), "v"(off), "s"(base) : "memory");
}
__device__ __forceinline__ void lds_dma4(const void *base, uint32_t off, uint32_t lds) {
    uint32_t saved;
    asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
                 "global_load_lds_dword %2, %3\n\ts_nop 0\n\ts_mov_b32 m0, %0"
                 : "=&s"(saved) : "s"(lds), "v"(off), "s"(base) : "memory");
}
__device__ __forceinline__ uint32_t lds_byte_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
// wait until at most N of this wave's vector memory operations are in
// flight and its LDS operations are done, then the workgroup barrier
template <int N>
__device__ __forceinline__ void wait_barrier() {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}


}  // namespace ring
}  // namespace vj
