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

// Segmented inclusive sum across the wave: segments are contiguous lane
// ranges and head is the first lane of this lane's segment; afterwards lane
// l holds the sum over lanes [head, l].  Row shifts 1, 2, 4, 8 scan the rows
// of 16; broadcasts of lane 15 (to rows 1, 3) and lane 31 (to rows 2, 3)
// join the rows.
template <int NV>
__device__ __forceinline__ void wave_segmented_scan(float (&m)[NV], int lane, int head) {
    const bool c1 = lane - 1 >= head, c2 = lane - 2 >= head, c4 = lane - 4 >= head, c8 = lane - 8 >= head;
    const bool c16 = (lane & ~15) - 1 >= head, c32 = 31 >= head;
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x111, 0xF>(m[k]); m[k] += c1 ? o : 0.0f; }
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x112, 0xF>(m[k]); m[k] += c2 ? o : 0.0f; }
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x114, 0xF>(m[k]); m[k] += c4 ? o : 0.0f; }
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x118, 0xF>(m[k]); m[k] += c8 ? o : 0.0f; }
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x142, 0xA>(m[k]); m[k] += c16 ? o : 0.0f; }
#pragma unroll
    for (int k = 0; k < NV; ++k) { const float o = dpp_mov<0x143, 0xC>(m[k]); m[k] += c32 ? o : 0.0f; }
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
