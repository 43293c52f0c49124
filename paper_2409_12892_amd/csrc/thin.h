// Pair passes of a thinned gradient cache (device code, included by thin.hip
// and persist.hip).
//
// The paper's limitations (section 4.4) propose shrinking the cache
// by keeping the per-splat gradients only for every 32nd splat along a ray
// and redoing the alpha blending inside those local windows.  A thinned
// cache (the raster's thin fill, lm_options.thin_window = K) keeps, per
// 64-pixel block of a tile, its active splats in depth order as pieces
// (segment, mask of the block's pixels the splat contributes to, mask of
// those whose alpha is clamped), and per pixel the blend state in front of
// its contributors 0, K, 2K, ...: the transmittance T and the colour S still
// to be blended from that contributor on.  No per-pair value is stored.
//
// A wave owns one block and a lane one pixel.  The wave walks the block's
// pieces in depth order; a lane whose bit is set re-blends its pair in
// float32 (eq. alpha-blending and the cached quantities of supplement A.2):
//     alpha = min(0.99, o exp(power)),   S -= c alpha T,
//     dC/dalpha = T c - S / (1 - alpha), T *= 1 - alpha,
// taking (T, S) from its next checkpoint at every K-th contributor (the
// checkpoint after the current one is loaded a window ahead).  The pair's
// Jacobian row is then the full cache's (apply.hip).  J p accumulates in the
// lane (its pixel's u); for J^T u each piece's nine moments are summed over
// the wave and kept per block in LDS, and the blocks' sums are added in
// block order when a segment chunk is written (deterministic).  Segments are
// staged in LDS chunk by chunk; a block's pieces ascend by segment, so a
// wave's walk continues across chunks.
#pragma once

#include <type_traits>

#include "proj_math.h"
#include "wave.h"

namespace lm {
namespace {

constexpr int kThinThreads = kTileBlocks * kWave;   // one wave per block
constexpr int kThinCap = 128;                       // segments staged per chunk (products)
constexpr int kThinGramCap = 32;                    // segments per chunk (Gram pass)
constexpr float kL2e = 1.4426950408889634f;

// Blend state of one lane's walk along its pixel's ray.
struct Walk {
    const float4* ckp;   // the pixel's checkpoints
    float4 nxt;          // checkpoint of the next window (loaded a window ahead)
    int ci;              // next checkpoint to load
    int rem;             // contributors left in the current window
    float T, S0, S1, S2;
    __device__ __forceinline__ void start(const float4* p, bool valid) {
        ckp = p;
        nxt = valid ? p[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        ci = 1;
        rem = 0;
        T = S0 = S1 = S2 = 0.0f;
    }
    // in front of the pixel's next contributor: enter a new window when due
    __device__ __forceinline__ void step(int K) {
        if (rem == 0) {
            T = nxt.x;
            S0 = nxt.y;
            S1 = nxt.z;
            S2 = nxt.w;
            nxt = ckp[ci++];   // at most one past the pixel's last checkpoint
            rem = K;
        }
        --rem;
    }
};

// The tile, its view and this lane's pixel.
struct ThinTile {
    int64_t t, sb, j0, j1, ib, HW;
    int nseg, wid;
    bool valid;
    float fx, fy;
    const float4* ckp;
    __device__ __forceinline__ ThinTile(const CacheView& c, int64_t tile) : t(tile) {
        const int tid = threadIdx.x, lane = __lane_id();
        wid = __builtin_amdgcn_readfirstlane(tid / kWave);
        const CamDev& cam = c.cams[c.tile_view[t]];
        const int64_t lt = t - cam.tile_base;
        const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
        const int tw_mask = c.TW - 1;
        const int bpr = c.TW >> 3;
        // the raster's pixel of this thread: 8x8 blocks when the tile is at
        // least 8 pixels each way, else 64 consecutive pixels
        const int pl = (c.TW >= 8 && c.TH >= 8)
                           ? (((wid / bpr) << 3) + (lane >> 3)) * c.TW + ((wid % bpr) << 3) + (lane & 7)
                           : wid * kBlockPix + lane;
        const int px = tx * c.TW + (pl & tw_mask), py = ty * c.TH + (pl >> c.tw_shift);
        valid = pl < c.TW * c.TH && px < cam.W && py < cam.H;
        HW = (int64_t)cam.W * cam.H;
        ib = 3 * cam.pix_base + (int64_t)py * cam.W + px;
        const int64_t pg = cam.pix_base + (int64_t)py * cam.W + px;
        fx = (float)(pl & tw_mask);
        fy = (float)(pl >> c.tw_shift);
        sb = c.tile_seg_off[t];
        nseg = (int)(c.tile_seg_off[t + 1] - sb);
        j0 = c.tile_pair_off[t];
        for (int b = 0; b < wid; ++b) j0 += c.tile_blk[t * kTileBlocks + b];
        j1 = j0 + c.tile_blk[t * kTileBlocks + wid];
        ckp = c.ck + c.tile_ck_off[t] + (valid ? c.pix_ck[pg] : 0u);
    }
};

// One re-blended pair: the splat's exponent term, alpha and dC/dalpha
// (g0 = mean - 0.5 and the conic scaled for exp2, g1.x the scaled C and
// g1.y the opacity, col the splat's colour).
struct Pair {
    float dx, dy, G, alpha, aT, D0, D1, D2;
    bool clamped;
};
__device__ __forceinline__ Pair reblend(Walk& W, int K, float fx, float fy, const float4& g0, const float4& g1,
                                        const float4& col, bool clamped) {
    Pair q;
    W.step(K);
    q.clamped = clamped;
    q.dx = fx - g0.x;
    q.dy = fy - g0.y;
    q.G = __builtin_amdgcn_exp2f(q.dx * (g0.z * q.dx + g0.w * q.dy) + g1.x * q.dy * q.dy);
    q.alpha = clamped ? 0.99f : g1.y * q.G;
    q.aT = q.alpha * W.T;
    W.S0 -= col.x * q.aT;
    W.S1 -= col.y * q.aT;
    W.S2 -= col.z * q.aT;
    const float r = 1.0f / (1.0f - q.alpha);
    q.D0 = W.T * col.x - W.S0 * r;
    q.D1 = W.T * col.y - W.S1 * r;
    q.D2 = W.T * col.z - W.S2 * r;
    W.T *= 1.0f - q.alpha;
    return q;
}

// staged splat of segment s: g0, g1 as the full cache's tile pass, then the
// tangent coefficients (J) and the colour
__device__ __forceinline__ void stage_splat(const CacheView& c, int64_t s, float4* row, const float* dyc,
                                            bool tangents) {
    const int64_t ss = c.seg_stride;
    row[0] = make_float4(c.seg_f[s] - 0.5f, c.seg_f[ss + s] - 0.5f, -0.5f * kL2e * c.seg_f[2 * ss + s],
                         -kL2e * c.seg_f[3 * ss + s]);
    float4 w1 = make_float4(-0.5f * kL2e * c.seg_f[4 * ss + s], c.seg_f[5 * ss + s], 0.0f, 0.0f);
    if (tangents) {
        const float* dy = dyc + (int64_t)c.seg_gv[s] * 9;
        w1.z = dy[0];
        w1.w = dy[1];
        row[2] = make_float4(dy[2], dy[3], dy[4], dy[5]);
        row[3] = make_float4(dy[6], dy[7], dy[8], 0.0f);
    }
    row[1] = w1;
    row[4] = make_float4(c.seg_f[6 * ss + s], c.seg_f[7 * ss + s], c.seg_f[8 * ss + s], 0.0f);
}

// gt: the tile's index over the batch (the subsets' tiles one after another)
template <int MODE>
__device__ __forceinline__ void thin_tile_body(const ApplyBatch& Bt, int64_t gt) {
    int bi = 0;
    while (bi + 1 < Bt.n && gt >= Bt.tile_off[bi + 1]) ++bi;
    const ApplyArgs& a = Bt.a[bi];
    if (a.stop && *a.stop) return;
    const CacheView& c = a.c;
    __shared__ float4 s_sg[kThinCap][5];
    __shared__ float s_mom[kTileBlocks][9][kThinCap];
    __shared__ double s_red[kTileBlocks];
    const ThinTile tl(c, gt - Bt.tile_off[bi]);
    const int tid = threadIdx.x, lane = __lane_id();
    const int K = c.thin_k;

    float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
    if (MODE == MODE_JT && tl.valid) {
        u0 = a.uin[tl.ib];
        u1 = a.uin[tl.ib + tl.HW];
        u2 = a.uin[tl.ib + 2 * tl.HW];
    }

    // one walk over the tile's segment chunks: J (u of this lane's pixel)
    // or J^T (moments per piece, summed over the wave)
    auto walk = [&](auto jt_tag) {
        constexpr bool JT = decltype(jt_tag)::value;
        Walk W;
        W.start(tl.ckp, tl.valid);
        int64_t j = tl.j0;
        for (int c0 = 0; c0 < tl.nseg; c0 += kThinCap) {
            const int cn = min(tl.nseg - c0, kThinCap);
            __syncthreads();
            for (int i = tid; i < cn; i += kThinThreads) stage_splat(c, tl.sb + c0 + i, s_sg[i], a.dyc, !JT);
            if (JT)
                for (int i = tid; i < kTileBlocks * 9 * kThinCap; i += kThinThreads) (&s_mom[0][0][0])[i] = 0.0f;
            __syncthreads();
            const uint32_t s_lo = (uint32_t)(tl.sb + c0), s_hi = s_lo + (uint32_t)cn;
            while (j < tl.j1) {
                const uint32_t sg = c.piece_seg[j];
                if (sg >= s_hi) break;
                const uint64_t mask = c.piece_mask[j], cm = c.piece_cmask[j];
                const int si = (int)(sg - s_lo);
                float m[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) m[k] = 0.0f;
                if ((mask >> lane) & 1ull) {
                    const float4 g0 = s_sg[si][0], g1 = s_sg[si][1], col = s_sg[si][4];
                    const Pair q = reblend(W, K, tl.fx, tl.fy, g0, g1, col, (cm >> lane) & 1ull);
                    if (!JT) {
                        const float4 g2 = s_sg[si][2], g3 = s_sg[si][3];
                        const float dal_f = q.alpha * (q.dx * (g1.z + g2.x * q.dx + g2.y * q.dy) +
                                                       q.dy * (g1.w + g2.z * q.dy)) + q.G * g2.w;
                        const float dal = q.clamped ? 0.0f : dal_f;
                        u0 += q.D0 * dal + q.aT * g3.x;
                        u1 += q.D1 * dal + q.aT * g3.y;
                        u2 += q.D2 * dal + q.aT * g3.z;
                    } else {
                        const float w = q.D0 * u0 + q.D1 * u1 + q.D2 * u2;
                        const float aw = q.clamped ? 0.0f : q.alpha * w;
                        const float awx = aw * q.dx, awy = aw * q.dy;
                        m[0] = awx;
                        m[1] = awy;
                        m[2] = awx * q.dx;
                        m[3] = awx * q.dy;
                        m[4] = awy * q.dy;
                        m[5] = q.clamped ? 0.0f : q.G * w;
                        m[6] = q.aT * u0;
                        m[7] = q.aT * u1;
                        m[8] = q.aT * u2;
                    }
                }
                if (JT) {
                    wave_segmented_scan<9>(m, lane, 0);
                    if (lane == kWave - 1) {
#pragma unroll
                        for (int k = 0; k < 9; ++k) s_mom[tl.wid][k][si] = m[k];
                    }
                }
                ++j;
            }
            if (JT) {
                __syncthreads();
                for (int i = tid; i < cn * 9; i += kThinThreads) {
                    const int si = i / 9, k = i - si * 9;
                    float sum = s_mom[0][k][si];
#pragma unroll
                    for (int b = 1; b < kTileBlocks; ++b) sum += s_mom[b][k][si];
                    a.gmom[(int64_t)c.seg_pos[tl.sb + c0 + si] * 9 + k] = sum;
                }
            }
        }
    };

    if (MODE & MODE_J) {
        walk(std::false_type{});
        // u of this pixel is complete: ||J p||^2 (sum w u^2 with residual
        // weights), the J output, and w . u for the J^T half
        double sq = 0.0;
        if (tl.valid) {
            float w0 = 1.0f, w1 = 1.0f, w2 = 1.0f;
            if (c.wres) {
                w0 = c.wres[tl.ib];
                w1 = c.wres[tl.ib + tl.HW];
                w2 = c.wres[tl.ib + 2 * tl.HW];
            }
            const float wu0 = c.wres ? u0 * w0 : u0, wu1 = c.wres ? u1 * w1 : u1, wu2 = c.wres ? u2 * w2 : u2;
            sq = (double)u0 * (double)wu0 + (double)u1 * (double)wu1 + (double)u2 * (double)wu2;
            if (MODE == MODE_J && a.uout) {
                a.uout[tl.ib] = u0;
                a.uout[tl.ib + tl.HW] = u1;
                a.uout[tl.ib + 2 * tl.HW] = u2;
            }
            u0 = wu0;
            u1 = wu1;
            u2 = wu2;
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sq += __shfl_xor(sq, off, kWave);
        if (lane == 0) s_red[tl.wid] = sq;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < kTileBlocks; ++w) tot += s_red[w];
            a.jp_part[tl.t] = tot;
        }
    }
    if (MODE & MODE_JT) walk(std::true_type{});
}

template <int MODE>
__global__ void __launch_bounds__(kThinThreads) k_thin_tile(ApplyBatch Bt) {
    thin_tile_body<MODE>(Bt, blockIdx.x);
}

}  // namespace
}  // namespace lm
