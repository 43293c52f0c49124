// Wave-level sums shared by the pair passes (apply.hip, thin.hip).
#pragma once

#include "lm_internal.h"

namespace lm {

// Data-parallel-primitive lane moves (VALU, no LDS): lanes whose source is
// outside the row or in a row not selected by ROWMASK read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}
// Row shift across all rows: lanes whose source is outside the row read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_shr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Segmented inclusive sum across the wave: segments are contiguous lane
// ranges and head is the first lane of this lane's segment; afterwards lane
// l holds the sum over lanes [head, l].  Row shifts 1, 2, 4, 8 scan the rows
// of 16; broadcasts of lane 15 (to rows 1, 3) and lane 31 (to rows 2, 3)
// join the rows.  Each step adds the moved value times a 0/1 factor (the
// lane's segment reaches that far back): an exact add or no change, in one
// multiply-add that takes the lane move as its operand.
template <int NV>
__device__ __forceinline__ void wave_segmented_scan(float (&m)[NV], int lane, int head) {
    const float c1 = lane - 1 >= head ? 1.0f : 0.0f, c2 = lane - 2 >= head ? 1.0f : 0.0f;
    const float c4 = lane - 4 >= head ? 1.0f : 0.0f, c8 = lane - 8 >= head ? 1.0f : 0.0f;
    const float c16 = (lane & ~15) - 1 >= head ? 1.0f : 0.0f, c32 = 31 >= head ? 1.0f : 0.0f;
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x111>(m[k]), c1, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x112>(m[k]), c2, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x114>(m[k]), c4, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x118>(m[k]), c8, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_mov<0x142, 0xA>(m[k]), c16, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_mov<0x143, 0xC>(m[k]), c32, m[k]);
}

// The same sum for segments of at most 8 lanes (a piece: one splat's pairs
// in one 64-pixel block, at most 8 runs of 8): row shifts 1, 2, 4 scan
// within the rows of 16, then a segment that starts in the previous row
// takes that row's last lane (lanes 15, 31, 47 to rows 1, 2, 3).  Lanes of
// a longer segment hold partial sums.
template <int NV>
__device__ __forceinline__ void wave_piece_scan(float (&m)[NV], int lane, int head) {
    const float c1 = lane - 1 >= head ? 1.0f : 0.0f, c2 = lane - 2 >= head ? 1.0f : 0.0f;
    const float c4 = lane - 4 >= head ? 1.0f : 0.0f, c16 = (lane & ~15) - 1 >= head ? 1.0f : 0.0f;
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x111>(m[k]), c1, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x112>(m[k]), c2, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_shr<0x114>(m[k]), c4, m[k]);
#pragma unroll
    for (int k = 0; k < NV; ++k) m[k] = __builtin_fmaf(dpp_mov<0x142, 0xE>(m[k]), c16, m[k]);
}

// First lane of this lane's segment, given per-lane segment keys that are
// ascending across the wave.
__device__ __forceinline__ int segment_head(uint32_t key, int lane) {
    const uint32_t prev = __shfl_up(key, 1, kWave);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
    return kWave - 1 - __clzll(heads & upto);
}

}  // namespace lm
