// Kernels of the thinned gradient cache (the device code is thin.h): the
// products and the per-segment Gram values, re-blending every pair.
#include "thin.h"

namespace lm {
namespace {

// Per-segment Gram values of a thinned cache (the full cache's k_gram_tile:
// per pair b = (alpha dx, alpha dy, alpha dx^2, alpha dx dy, alpha dy^2, G)
// (zero when alpha is clamped), e = alpha T, D = dC/dalpha; Bbb, Ebd, E2
// and the pair count), summed per piece over the wave, per segment over the
// blocks in block order.
__global__ void __launch_bounds__(kThinThreads) k_thin_gram(CacheView c, float* __restrict__ gram) {
    constexpr int NG = kGramValues;
    __shared__ float4 s_sg[kThinGramCap][5];
    __shared__ float s_g[kTileBlocks][NG][kThinGramCap];
    const ThinTile tl(c, blockIdx.x);
    const int tid = threadIdx.x, lane = __lane_id();
    const int K = c.thin_k;
    float w0 = 1.0f, w1 = 1.0f, w2 = 1.0f;
    if (c.wres && tl.valid) {
        w0 = c.wres[tl.ib];
        w1 = c.wres[tl.ib + tl.HW];
        w2 = c.wres[tl.ib + 2 * tl.HW];
    }
    Walk W;
    W.start(tl.ckp, tl.valid);
    int64_t j = tl.j0;
    for (int c0 = 0; c0 < tl.nseg; c0 += kThinGramCap) {
        const int cn = min(tl.nseg - c0, kThinGramCap);
        __syncthreads();
        for (int i = tid; i < cn; i += kThinThreads) stage_splat(c, tl.sb + c0 + i, s_sg[i], nullptr, false);
        for (int i = tid; i < kTileBlocks * NG * kThinGramCap; i += kThinThreads) (&s_g[0][0][0])[i] = 0.0f;
        __syncthreads();
        const uint32_t s_lo = (uint32_t)(tl.sb + c0), s_hi = s_lo + (uint32_t)cn;
        while (j < tl.j1) {
            const uint32_t sg = c.piece_seg[j];
            if (sg >= s_hi) break;
            const uint64_t mask = c.piece_mask[j], cm = c.piece_cmask[j];
            const int si = (int)(sg - s_lo);
            float acc[NG];
#pragma unroll
            for (int k = 0; k < NG; ++k) acc[k] = 0.0f;
            if ((mask >> lane) & 1ull) {
                const Pair q = reblend(W, K, tl.fx, tl.fy, s_sg[si][0], s_sg[si][1], s_sg[si][4], (cm >> lane) & 1ull);
                const float ag = q.clamped ? 0.0f : q.alpha;
                float bb[6];
                bb[0] = ag * q.dx;
                bb[1] = ag * q.dy;
                bb[2] = ag * q.dx * q.dx;
                bb[3] = ag * q.dx * q.dy;
                bb[4] = ag * q.dy * q.dy;
                bb[5] = q.clamped ? 0.0f : q.G;
                const float WD0 = w0 * q.D0, WD1 = w1 * q.D1, WD2 = w2 * q.D2;
                const float DD = WD0 * q.D0 + WD1 * q.D1 + WD2 * q.D2;
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int k = i; k < 6; ++k) acc[i * 6 - (i * (i - 1)) / 2 + (k - i)] = DD * bb[i] * bb[k];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const float eb = q.aT * bb[i];
                    acc[21 + 3 * i] = eb * WD0;
                    acc[22 + 3 * i] = eb * WD1;
                    acc[23 + 3 * i] = eb * WD2;
                }
                const float ee = q.aT * q.aT;
                acc[39] = w0 * ee;
                acc[40] = w1 * ee;
                acc[41] = w2 * ee;
                acc[42] = 1.0f;
            }
            wave_segmented_scan<NG>(acc, lane, 0);
            if (lane == kWave - 1) {
#pragma unroll
                for (int k = 0; k < NG; ++k) s_g[tl.wid][k][si] = acc[k];
            }
            ++j;
        }
        __syncthreads();
        for (int i = tid; i < cn * NG; i += kThinThreads) {
            const int si = i / NG, k = i - si * NG;
            float sum = s_g[0][k][si];
#pragma unroll
            for (int b = 1; b < kTileBlocks; ++b) sum += s_g[b][k][si];
            gram[(int64_t)c.seg_pos[tl.sb + c0 + si] * NG + k] = sum;
        }
    }
}

}  // namespace

hipError_t launch_thin_tile(int mode, const ApplyBatch& B, hipStream_t s) {
    const int64_t nt = B.tile_off[B.n];
    if (nt == 0) return hipSuccess;
    const dim3 g((unsigned)nt), b(kThinThreads);
    if (mode == MODE_J) hipLaunchKernelGGL(k_thin_tile<MODE_J>, g, b, 0, s, B);
    else if (mode == MODE_JT) hipLaunchKernelGGL(k_thin_tile<MODE_JT>, g, b, 0, s, B);
    else hipLaunchKernelGGL(k_thin_tile<MODE_JTJ>, g, b, 0, s, B);
    return hipGetLastError();
}

hipError_t launch_thin_gram(const CacheView& c, float* gram, hipStream_t s) {
    if (c.n_tiles == 0 || c.n_seg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_thin_gram, dim3((unsigned)c.n_tiles), dim3(kThinThreads), 0, s, c, gram);
    return hipGetLastError();
}

}  // namespace lm
