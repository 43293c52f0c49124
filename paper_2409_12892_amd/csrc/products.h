// Product passes of the gradient cache (paper section 3.3 and supplement A):
// u = J p (eq. apply-j), g = J^T u (eq. apply-jt) and the fused
// (J^T J + lambda M) p of Algorithm 1.  Every pass is a device body, run by
// its own kernel (apply.hip) or by the persistent PCG kernel (persist.hip).
//
// The Jacobian of a pixel colour with respect to the splat attributes y of
// one contributing splat (the middle factor of eq. backward-pass) is
//     dC_ch/dy = [ D_ch dalpha/dy_geo  |  alpha T e_ch ]
// with D = dC/dalpha and T read from the cache and alpha, dalpha/dy_geo
// recomputed from the staged splat (mean, conic, opacity) and the pixel.
// The splat-to-parameter factor dy/dx is applied per (Gaussian, view): the
// projection is linearised once per cache (float64, stored as float32), the
// tangent maps p through it to per-(Gaussian, view) power coefficients
// before the tile pass, and the chain applies its transpose to the
// per-(Gaussian, view) moments after it (supplement A.2 splits applyJT the
// same way).
//
// Tile pass: one workgroup of 512 threads per tile.  A tile's pairs are
// stored block by block (a block is the 64 pixels of one raster wave);
// within a block the active splats in depth order, each with its pairs in
// the block (a piece) padded to whole runs of 8 pairs, and no piece crosses
// a window of 512 pairs from the block's start, so a wave that takes a
// window's 64 runs (one per lane) sums every piece it sees completely.
//   J  : lanes add the J rows of their runs into per-wave LDS accumulators
//        of the block's pixels; the waves' accumulators are added in wave
//        order, which completes u for the block.
//   J^T: the same runs (held in registers by the fused pass, so each pair is
//        read once) give 9 moments per lane; a segmented scan over the wave
//        leaves one LDS addition per piece, i.e. per segment and block, in
//        block order (deterministic).
// Runs past the register capacity are streamed in each half, and tiles with
// more segments than one LDS stage holds run chunk by chunk.  u stays in
// LDS between the halves (every pixel's splats live in its own tile).
#pragma once

#include <algorithm>

#include "proj_math.h"
#include "wave.h"

namespace lm {
namespace {

constexpr int kRun = 8;        // pairs per run (pieces are padded to runs)
constexpr int kWinRuns = kWindow / kRun;   // runs of a wave's window (no piece crosses one)


// One aligned run of 8 pairs as loaded: the words kept packed as loaded
// (two 16-bit words per register for the 16-bit caches, four pixel bytes
// per register), unpacked where used.
template <int DT>
struct RunLoad {
    using S = Store<DT>;
    using W = typename S::word;
    static constexpr int NWD = kRun * (int)sizeof(W) / 4;   // 32-bit registers per plane
    uint32_t tw[NWD];
    uint32_t dw[3][NWD];
    uint32_t pw[2];
    uint32_t seg;
    __device__ __forceinline__ W word(const uint32_t* p, int k) const {
        if constexpr (sizeof(W) == 4) return p[k];
        else return (W)((p[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
    }
    __device__ __forceinline__ W t(int k) const { return word(tw, k); }
    __device__ __forceinline__ W d(int ch, int k) const { return word(dw[ch], k); }
    __device__ __forceinline__ int pix(int k) const { return (int)((pw[k >> 2] >> (8 * (k & 3))) & 0xFFu); }
};

// ---- linearisation: the projection of every (Gaussian, view) at x ----------
// Columns of the tangent map (unit tangents of the 11 geometric parameters)
// in float64, stored as float32; the SH part is the basis itself.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_linearize(CacheView c, const float* __restrict__ x,
                                                     float* __restrict__ lin) {
    const int64_t gv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gv >= c.n_gv) return;
    const uint32_t rec = c.gv_rec[gv];
    const int v = (int)(rec / c.N);
    const int64_t g = rec - (int64_t)v * c.N;
    const CamDev& cam = c.cams[v];
    ProjFwd f;
    proj_forward<DEG>(cam, x, c.N, g, f);
    const int64_t ls = c.lin_stride;
#pragma unroll 1
    for (int j = 0; j < 11; ++j) {
        double unit[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) unit[i] = i == j ? 1.0 : 0.0;
        double co[9];
        proj_tangent<DEG>(cam, f, unit, x, nullptr, c.N, g, co);
#pragma unroll
        for (int i = 0; i < 6; ++i) lin[(int64_t)(kLinL + 11 * i + j) * ls + gv] = (float)co[i];
        if (j < 3) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) lin[(int64_t)(kLinJdir + 3 * ch + j) * ls + gv] = (float)co[6 + ch];
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) lin[(int64_t)(kLinY + k) * ls + gv] = k < (DEG + 1) * (DEG + 1) ? (float)f.Y[k] : 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) lin[(int64_t)(kLinMask + ch) * ls + gv] = f.clamp[ch] ? 0.0f : 1.0f;
}

// ---- tangent: p -> per-(Gaussian, view) power coefficients -------------------
template <int DEG>
__device__ __forceinline__ void tangent_body(const ApplyArgs& a, int64_t gv) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const CacheView& c = a.c;
    if (gv >= c.n_gv) return;
    const int64_t g = c.gv_rec[gv] % (uint32_t)c.N;
    const int64_t ls = c.lin_stride, N = c.N;
    float dgeo[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) dgeo[j] = a.p[(int64_t)j * N + g];
    float out[9];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 11; ++j) acc += (double)c.lin[(int64_t)(kLinL + 11 * i + j) * ls + gv] * (double)dgeo[j];
        out[i] = (float)acc;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) acc += (double)c.lin[(int64_t)(kLinJdir + 3 * ch + m) * ls + gv] * (double)dgeo[m];
        double sh = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            sh += (double)c.lin[(int64_t)(kLinY + k) * ls + gv] * (double)a.p[(int64_t)(11 + 3 * k + ch) * N + g];
        out[6 + ch] = (float)(acc + (double)c.lin[(int64_t)(kLinMask + ch) * ls + gv] * sh);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) a.dyc[gv * 9 + k] = out[k];
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_tangent(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    tangent_body<DEG>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---- pair pass ---------------------------------------------------------------
// Per pair, with the splat staged in LDS: alpha and dalpha/dy are recomputed
// from the pixel position and the cached T, dC/dalpha give
//   J row block . dy = D (dalpha/dy_geo . a) + alpha T dc      (a: power coefficients)
// The staged splat holds the mean shifted to pixel-centre coordinates and
// the conic scaled by -log2(e)/2 (and -log2(e) for B), so exp(power) is one
// exp2 of a quadratic form.
constexpr float kLog2e = 1.4426950408889634f;

// Buffer resources over one tile's slots: every plane is addressed by a
// 32-bit tile-local offset from a base held in scalar registers, and a read
// past the tile's last slot returns 0 (a zero T word is no pair), so the
// per-lane loads need neither 64-bit address arithmetic nor a bounds test.
// A tile holds at most 256 pixels x ~2350 blended splats plus padding, far
// below the 2 GB range of a resource.
constexpr int kRsrcWord3 = 0x00020000;

template <int DT>
struct TilePlanes {
    using W = typename Store<DT>::word;
    __amdgpu_buffer_rsrc_t t, d0, d1, d2, pix, seg;
    __device__ __forceinline__ TilePlanes(const CacheView& c, int64_t pb, int64_t pe) {
        const int n = (int)(pe - pb);
        const int nb = n * (int)sizeof(W);
        const W* pt = (const W*)c.pT + pb;
        const W* pd = (const W*)c.pD + pb;
        t = __builtin_amdgcn_make_buffer_rsrc((void*)pt, (short)0, nb, kRsrcWord3);
        d0 = __builtin_amdgcn_make_buffer_rsrc((void*)pd, (short)0, nb, kRsrcWord3);
        d1 = __builtin_amdgcn_make_buffer_rsrc((void*)(pd + c.pair_stride), (short)0, nb, kRsrcWord3);
        d2 = __builtin_amdgcn_make_buffer_rsrc((void*)(pd + 2 * c.pair_stride), (short)0, nb, kRsrcWord3);
        pix = __builtin_amdgcn_make_buffer_rsrc((void*)(c.ppix + pb), (short)0, n, kRsrcWord3);
        seg = __builtin_amdgcn_make_buffer_rsrc((void*)(c.run_seg + pb / kRun), (short)0, (n / kRun) * 4,
                                                kRsrcWord3);
    }
    __device__ __forceinline__ W word(__amdgpu_buffer_rsrc_t r, int q) const {
        if constexpr (sizeof(W) == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, q * 4, 0, 0);
        else return __builtin_amdgcn_raw_buffer_load_b16(r, q * 2, 0, 0);
    }
    // aligned run r of the tile when `want`; otherwise a run index past
    // every tile (the buffer range check returns zeros without a memory
    // access) and a segment word no chunk holds.  Straight-line, so the
    // run stays in registers.
    __device__ __forceinline__ void run_if(int r, RunLoad<DT>& L, bool want) const {
        run(want ? r : (1 << 24), L);
        L.seg = want ? L.seg : 0xFFFFFFFFu;
    }
    // aligned run r of the tile (eight pairs per lane)
    __device__ __forceinline__ void run(int r, RunLoad<DT>& L) const {
        L.seg = __builtin_amdgcn_raw_buffer_load_b32(seg, r * 4, 0, 0);
        constexpr int NWD = RunLoad<DT>::NWD;
        const int o = r * NWD * 4;
        const __amdgpu_buffer_rsrc_t pr[4] = {t, d0, d1, d2};
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
            uint32_t* dst = pl == 0 ? L.tw : L.dw[pl - 1];
#pragma unroll
            for (int h = 0; h < NWD / 4; ++h) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(pr[pl], o + 16 * h, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[4 * h + i] = v[i];
            }
        }
        const auto px = __builtin_amdgcn_raw_buffer_load_b64(pix, r * kRun, 0, 0);
        L.pw[0] = px[0];
        L.pw[1] = px[1];
    }
};

// First run in [lo, hi) of a tile whose segment word is >= key (hi if
// none), for runs whose segments ascend (a block's runs: pieces in segment
// order, a gap run carrying the next piece's segment).  The wave probes 64
// runs at a time, so a block of up to 2^18 runs takes three rounds of
// dependent loads.  Wave-uniform arguments; every lane returns the result.
__device__ __forceinline__ int run_lower_bound(__amdgpu_buffer_rsrc_t seg, int lo, int hi, uint32_t key, int lane) {
    while (hi > lo) {
        const int step = (hi - lo + kWave - 1) / kWave;
        const int r = lo + lane * step;
        const bool ge = r >= hi || __builtin_amdgcn_raw_buffer_load_b32(seg, r * 4, 0, 0) >= key;
        const uint64_t m = __ballot(ge);
        // runs before the first probe at or above the key are below it
        const int f = m ? __ffsll((unsigned long long)m) - 1 : kWave;
        if (step == 1) {
            lo = hi = min(hi, lo + f);
        } else {
            const int nlo = f == 0 ? lo : lo + (f - 1) * step + 1;
            hi = min(hi, lo + f * step);
            lo = nlo;
        }
    }
    return lo;
}

// Tile pass.  One workgroup of 512 threads (8 waves) per tile.  The tile's
// pairs are stored block after block (a block is the 64 pixels of one
// raster wave); within a block the splats' pieces in segment order, each
// padded to whole runs of 8 pairs, and no piece crosses a window of 512
// pairs from its block's start.
//   J  : the tile's pairs in windows of 64, one pair per lane (coalesced
//        loads), window k by wave k mod 8 (balanced to one window), two
//        groups of kJGroup windows in flight per wave.  Per window the J
//        rows of the lanes' pairs; the window's pieces (contiguous lane
//        ranges with distinct pixels; a segment's pieces of two adjacent
//        blocks have distinct pixels too) add into the wave's per-pixel
//        accumulators one after another with plain LDS read-modify-writes.
//        The waves' accumulators are added in wave order into u.
//   J^T: block by block, the block's 512-pair windows in run order (64 runs
//        of 8 pairs, one per lane; a run belongs to one piece), window c by
//        wave c mod 8.  Each lane sums the 9 moments of its run, one
//        segmented scan over the wave (keyed by segment) leaves each
//        piece's sum in its last lane, which adds it into the segment's
//        moments: a segment has one piece per block, in one window, so one
//        wave adds per block, and a barrier between blocks orders the
//        additions.
// No LDS atomics, and every sum runs in a fixed order.  A tile with more
// segments than LDS stages at once (kSegCap) runs segment chunk after
// segment chunk.
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kSegCap = 640;
constexpr int kChunkRuns = kWave;                 // runs of a J^T window (one per lane)
static_assert(kChunkRuns * kRun == kWindow, "a J^T window is one placement window");
constexpr int kJGroup = 4;                        // 64-pair J windows a wave loads together

// A group of J windows in pair order: window j's word of lane l is pair
// 64 j + l of the group; 16-bit words two per register, pixel bytes four
// per register, segment words one per window.
template <int DT>
struct PairGroup {
    using S = Store<DT>;
    using W = typename S::word;
    static constexpr int NR = sizeof(W) == 4 ? kJGroup : kJGroup / 2;   // registers per plane
    uint32_t tw[NR];
    uint32_t dw[3][NR];
    uint32_t pw[(kJGroup + 3) / 4];
    uint32_t sg[kJGroup];
    int lim[kJGroup];                 // pairs of window j in its range (wave-uniform)
    __device__ __forceinline__ W word(const uint32_t* p, int j) const {
        if constexpr (sizeof(W) == 4) return p[j];
        else return (W)((p[j >> 1] >> (16 * (j & 1))) & 0xFFFFu);
    }
    __device__ __forceinline__ W t(int j) const { return word(tw, j); }
    __device__ __forceinline__ W d(int ch, int j) const { return word(dw[ch], j); }
    __device__ __forceinline__ int pix(int j) const { return (int)((pw[j >> 2] >> (8 * (j & 3))) & 0xFFu); }
};

// J windows: window j of the group starts at tile-relative pair q0[j] and
// holds lim[j] pairs of its range (a window past the tile reads zeros
// without a memory access)
template <int DT>
__device__ __forceinline__ void load_pair_group(const TilePlanes<DT>& P, const int (&q0)[kJGroup], int lane,
                                                PairGroup<DT>& L) {
    using W = typename Store<DT>::word;
    const __amdgpu_buffer_rsrc_t pr[4] = {P.t, P.d0, P.d1, P.d2};
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
        uint32_t* dst = pl == 0 ? L.tw : L.dw[pl - 1];
#pragma unroll
        for (int j = 0; j < kJGroup; ++j) {
            const int q = q0[j] + lane;
            if constexpr (sizeof(W) == 4) {
                dst[j] = __builtin_amdgcn_raw_buffer_load_b32(pr[pl], q * 4, 0, 0);
            } else {
                const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(pr[pl], q * 2, 0, 0);
                dst[j >> 1] = (j & 1) ? (dst[j >> 1] | (h << 16)) : h;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kJGroup; ++j) {
        const uint32_t q = (uint32_t)(q0[j] + lane);
        const uint32_t b = __builtin_amdgcn_raw_buffer_load_b8(P.pix, (int)q, 0, 0);
        L.pw[j >> 2] = (j & 3) ? (L.pw[j >> 2] | (b << (8 * (j & 3)))) : b;
        L.sg[j] = __builtin_amdgcn_raw_buffer_load_b32(P.seg, (int)((q >> 3) << 2), 0, 0);
    }
}

// gt: the tile's index over the batch (the subsets' tiles one after another)
template <int MODE, int DT>
__device__ __forceinline__ void apply_tile_body(const ApplyBatch& Bt, int64_t gt) {
    int bi = 0;
    while (bi + 1 < Bt.n && gt >= Bt.tile_off[bi + 1]) ++bi;
    const ApplyArgs& a = Bt.a[bi];
    if (a.stop && *a.stop) return;
    using S = Store<DT>;
    constexpr int NW = kTileWaves;
    constexpr int kNoSeg = kSegCap;              // segment key of a lane without a run
    const CacheView& c = a.c;
    __shared__ float4 s_sg[kSegCap][4];   // mx', my', A', B' | C', o, P1, P2 | Q1, Q2, Q3, do | dc0, dc1, dc2, -
    // the J half's per-wave accumulators (u of each pixel, w unused) and the
    // J^T half's segment moments share their LDS (the halves run one after
    // the other)
    constexpr int kAcc = 4 * NW * kMaxTilePix > 9 * kSegCap ? 4 * NW * kMaxTilePix : 9 * kSegCap;
    __shared__ __align__(16) float s_acc[kAcc];
    float4 (*s_uw)[kMaxTilePix] = reinterpret_cast<float4 (*)[kMaxTilePix]>(s_acc);
    float (*s_mom)[kSegCap] = reinterpret_cast<float (*)[kSegCap]>(s_acc);
    __shared__ float4 s_ut[kMaxTilePix];        // u of the tile (weighted once complete)
    __shared__ double s_red[NW];
    __shared__ int br[kTileBlocks + 1];         // tile-relative first run of each block
    __shared__ int rng[kTileBlocks][2];         // runs of the staged segments in each block
    __shared__ int wpre[kTileBlocks + 1];       // J windows of the blocks' ranges before each block

    const int64_t t = gt - Bt.tile_off[bi];
    const int tid = threadIdx.x, lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int v = c.tile_view[t];
    const CamDev& cam = c.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
    const int tw_mask = c.TW - 1, tw_shift = c.tw_shift;
    const int npix = c.TW * c.TH;
    const int nblk = (npix + kBlockPix - 1) / kBlockPix;
    const int64_t HW = (int64_t)cam.W * cam.H;
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    const int nseg = (int)(se - sb);
    const TilePlanes<DT> P(c, pb, pe);
    if (tid == 0) {
        br[0] = 0;
#pragma unroll
        for (int b = 0; b < kTileBlocks; ++b) br[b + 1] = br[b] + (int)c.tile_blk[t * kTileBlocks + b] / kRun;
    }

    auto pix_valid = [&](int pl) -> bool {
        return pl < npix && tx * c.TW + (pl & tw_mask) < cam.W && ty * c.TH + (pl >> tw_shift) < cam.H;
    };
    auto img_index = [&](int pl) -> int64_t {
        return 3 * cam.pix_base + (int64_t)(ty * c.TH + (pl >> tw_shift)) * cam.W + tx * c.TW + (pl & tw_mask);
    };

    for (int i = tid; i < kMaxTilePix; i += kTileThreads) s_ut[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (MODE & MODE_J)
        for (int i = tid; i < 4 * NW * kMaxTilePix; i += kTileThreads) s_acc[i] = 0.0f;
    __syncthreads();
    if (MODE == MODE_JT && tid < npix && pix_valid(tid)) {
        const int64_t ib = img_index(tid);
        s_ut[tid] = make_float4(a.uin[ib], a.uin[ib + HW], a.uin[ib + 2 * HW], 0.0f);
    }

    // segments [c0, c0 + cn): splat data (and tangents) into LDS
    auto stage = [&](int c0, int cn, bool tangents) {
        for (int i = tid; i < cn; i += kTileThreads) {
            const int64_t s = sb + c0 + i;
            const int64_t ss = c.seg_stride;
            s_sg[i][0] = make_float4(c.seg_f[s] - 0.5f, c.seg_f[ss + s] - 0.5f, -0.5f * kLog2e * c.seg_f[2 * ss + s],
                                     -kLog2e * c.seg_f[3 * ss + s]);
            float4 w1 = make_float4(-0.5f * kLog2e * c.seg_f[4 * ss + s], c.seg_f[5 * ss + s], 0.0f, 0.0f);
            if (tangents) {
                const float* dy = a.dyc + (int64_t)c.seg_gv[s] * 9;
                w1.z = dy[0];
                w1.w = dy[1];
                s_sg[i][2] = make_float4(dy[2], dy[3], dy[4], dy[5]);
                s_sg[i][3] = make_float4(dy[6], dy[7], dy[8], 0.0f);
            }
            s_sg[i][1] = w1;
        }
    };
    auto zero_mom = [&](int cn) {
        for (int i = tid; i < cn; i += kTileThreads)
#pragma unroll
            for (int k = 0; k < 9; ++k) s_mom[k][i] = 0.0f;
    };

    // J rows of one group of windows (segments [s0, s0 + cn) staged) into
    // this wave's accumulators
    auto j_group = [&](const PairGroup<DT>& L, int64_t s0, int cn) {
        float4* uw = s_uw[wid];
#pragma unroll
        for (int j = 0; j < kJGroup; ++j) {
            const uint32_t sg = L.sg[j];
            const uint32_t sl = sg - (uint32_t)s0;        // segment ids fit 32 bits
            const bool live = lane < L.lim[j] && L.t(j) != 0 && sl < (uint32_t)cn;
            float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
            const int pl = L.pix(j);
            if (live) {
                const int s = (int)sl;
                const float4 g0 = s_sg[s][0], g1 = s_sg[s][1], g2 = s_sg[s][2], g3 = s_sg[s][3];
                const float T = S::dec_T(L.t(j));
                const bool clamped = S::clamp(L.t(j));
                const float dx = (float)(pl & tw_mask) - g0.x;
                const float dy = (float)(pl >> tw_shift) - g0.y;
                const float G = __builtin_amdgcn_exp2f(dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy);
                const float alpha = clamped ? 0.99f : g1.y * G;
                const float aT = alpha * T;
                const float dal_f = alpha * (dx * (g1.z + g2.x * dx + g2.y * dy) + dy * (g1.w + g2.z * dy)) + G * g2.w;
                const float dal = clamped ? 0.0f : dal_f;
                v0 = S::dec(L.d(0, j)) * dal + aT * g3.x;
                v1 = S::dec(L.d(1, j)) * dal + aT * g3.y;
                v2 = S::dec(L.d(2, j)) * dal + aT * g3.z;
            }
            // the window's pieces one after another (pixels are distinct
            // within a segment's pieces)
            const uint64_t livem = __ballot(live);
            uint64_t todo = livem;
            while (todo) {
                const int first = __ffsll((unsigned long long)todo) - 1;
                const uint32_t sk = (uint32_t)__builtin_amdgcn_readlane((int)sg, first);
                const bool same = sg == sk;
                todo &= ~(__ballot(same) & livem);
                if (same && live) {
                    float4 u = uw[pl];
                    u.x += v0;
                    u.y += v1;
                    u.z += v2;
                    uw[pl] = u;
                }
            }
        }
    };
    // the runs of segments [s_lo, s_hi) (global ids) in each block into
    // rng (each bound a lower bound over the block's run segments, by wave
    // 2 b + e), and the J windows of those ranges into wpre
    auto find_ranges = [&](int64_t s_lo, int64_t s_hi, bool whole) {
        if (whole) {
            if (tid < kTileBlocks) {
                rng[tid][0] = br[tid];
                rng[tid][1] = br[tid + 1];
            }
        } else if (wid < 2 * kTileBlocks) {
            const int b = wid >> 1;
            const uint32_t key = (uint32_t)((wid & 1) ? s_hi : s_lo);
            const int r = run_lower_bound(P.seg, br[b], br[b + 1], key, lane);
            if (lane == 0) rng[b][wid & 1] = r;
        }
        __syncthreads();
        if (tid == 0) {
            wpre[0] = 0;
#pragma unroll
            for (int b = 0; b < kTileBlocks; ++b) wpre[b + 1] = wpre[b] + (rng[b][1] - rng[b][0] + 7) / 8;
        }
        __syncthreads();
    };
    // start pair and pair count of J window i (past the last: none)
    auto window = [&](int i, int& q0, int& lim) {
        int b = 0;
#pragma unroll
        for (int k = 1; k < kTileBlocks; ++k) b = i >= wpre[k] ? k : b;
        if (i >= wpre[kTileBlocks]) {
            q0 = 1 << 28;
            lim = 0;
        } else {
            q0 = rng[b][0] * kRun + (i - wpre[b]) * kWave;
            lim = min(kWave, rng[b][1] * kRun - q0);
        }
    };
    auto load_windows = [&](int i0, PairGroup<DT>& L) {
        int q0[kJGroup];
#pragma unroll
        for (int j = 0; j < kJGroup; ++j) window(i0 + j * NW, q0[j], L.lim[j]);
        load_pair_group(P, q0, lane, L);
    };
    // this wave's J windows of the ranges, segments [s0, s0 + cn) staged;
    // two groups in flight
    auto j_tile = [&](int64_t s0, int cn) {
        const int nw = wpre[kTileBlocks];
        PairGroup<DT> cur, nxt;
        load_windows(wid, cur);
        for (int i0 = wid; i0 < nw; i0 += kJGroup * NW) {
            load_windows(i0 + kJGroup * NW, nxt);
            j_group(cur, s0, cn);
            cur = nxt;
        }
    };
    // u of the tile: the waves' accumulators in wave order; ||J p||^2 (sum
    // w u^2 with residual weights), the J output, and w . u for J^T
    double sq = 0.0;
    auto finish_u = [&] {
        for (int pl = tid; pl < npix; pl += kTileThreads) {
            float4 u = s_uw[0][pl];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                const float4 o = s_uw[w][pl];
                u.x += o.x;
                u.y += o.y;
                u.z += o.z;
            }
            float4 wu = u;
            if (pix_valid(pl)) {
                const int64_t ib = img_index(pl);
                if (c.wres) {
                    wu.x = u.x * c.wres[ib];
                    wu.y = u.y * c.wres[ib + HW];
                    wu.z = u.z * c.wres[ib + 2 * HW];
                }
                sq += (double)u.x * (double)wu.x + (double)u.y * (double)wu.y + (double)u.z * (double)wu.z;
                if (MODE == MODE_J && a.uout) {
                    a.uout[ib] = u.x;
                    a.uout[ib + HW] = u.y;
                    a.uout[ib + 2 * HW] = u.z;
                }
            }
            s_ut[pl] = wu;
        }
    };

    // J^T moments of one window (lane: one run, segments [s0, s0 + cn)
    // staged): per lane the sums over its run, a segmented scan over the
    // wave, one plain addition per piece with pairs (a gap run carries the
    // next piece's segment and no pair: a group of gap runs adds nothing)
    auto jt_chunk = [&](const RunLoad<DT>& L, int64_t s0, int cn) {
        const uint32_t sl = L.seg - (uint32_t)s0;     // segment ids fit 32 bits
        const bool in = sl < (uint32_t)cn;
        const int key = in ? (int)sl : kNoSeg;
        float m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = 0.0f;
        // a run with pairs has a nonzero T word (a stored T is at least 1e-4)
        uint32_t tor = 0u;
#pragma unroll
        for (int i = 0; i < RunLoad<DT>::NWD; ++i) tor |= L.tw[i];
        const bool any = tor != 0u && in;
        {
            const int s = in ? key : 0;
            const float4 g0 = s_sg[s][0], g1 = s_sg[s][1];
            // a padding pair has T, D and pixel 0: w = D . u and alpha T are
            // 0, so every term is 0 (G and alpha are finite: the power is
            // <= 0; u is pixel 0's, finite); lanes outside [s0, s0 + cn) sum
            // under a key no piece has
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const float T = S::dec_T(L.t(k));
                const bool clamped = S::clamp(L.t(k));
                const int pl = L.pix(k);
                const float dx = (float)(pl & tw_mask) - g0.x;
                const float dy = (float)(pl >> tw_shift) - g0.y;
                const float G = __builtin_amdgcn_exp2f(dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy);
                const float alpha = clamped ? 0.99f : g1.y * G;
                const float aT = alpha * T;
                const float4 u = s_ut[pl];
                const float w = S::dec(L.d(0, k)) * u.x + S::dec(L.d(1, k)) * u.y + S::dec(L.d(2, k)) * u.z;
                const float aw = clamped ? 0.0f : alpha * w;
                const float awx = aw * dx, awy = aw * dy;
                m[0] += awx;
                m[1] += awy;
                m[2] += awx * dx;
                m[3] += awx * dy;
                m[4] += awy * dy;
                m[5] += clamped ? 0.0f : G * w;
                m[6] += aT * u.x;
                m[7] += aT * u.y;
                m[8] += aT * u.z;
            }
        }
        const uint64_t lives = __ballot(any);
        const int next = __shfl_down(key, 1, kWave);
        const int head = segment_head((uint32_t)key, lane);
        wave_piece_scan<9>(m, lane, head);
        const uint64_t grp = ((2ull << lane) - 1ull) & ~((1ull << head) - 1ull);
        if (key != kNoSeg && (lane == kWave - 1 || next != key) && (lives & grp) != 0ull) {
#pragma unroll
            for (int k = 0; k < 9; ++k) s_mom[k][key] += m[k];
        }
    };
    // the block's runs in a lane: run r of the 512-pair window ch of block b
    // when it lies in the block's range
    auto load_run_chunk = [&](int b, int ch, RunLoad<DT>& L) {
        const int r = br[b] + ch * kChunkRuns + lane;
        P.run_if(r, L, r >= rng[b][0] && r < rng[b][1]);
    };
    // the block's 512-pair windows that meet its range: [first, end)
    auto first_chunk = [&](int b) { return (rng[b][0] - br[b]) / kChunkRuns; };
    auto end_chunk = [&](int b) { return (rng[b][1] - br[b] + kChunkRuns - 1) / kChunkRuns; };
    // every block's J^T windows, blocks in order with a barrier after each
    // (the next block's first window of this wave loads meanwhile)
    auto jt_tile = [&](int64_t s0, int cn) {
        RunLoad<DT> nx;
        load_run_chunk(0, first_chunk(0) + wid, nx);
        for (int b = 0; b < nblk; ++b) {
            const int c_lo = first_chunk(b), c_hi = end_chunk(b);
            RunLoad<DT> cur = nx;
            if (b + 1 < nblk) load_run_chunk(b + 1, first_chunk(b + 1) + wid, nx);
            if (c_lo + wid < c_hi) jt_chunk(cur, s0, cn);
            for (int ch = c_lo + wid + NW; ch < c_hi; ch += NW) {
                RunLoad<DT> L;
                load_run_chunk(b, ch, L);
                jt_chunk(L, s0, cn);
            }
            __syncthreads();
        }
    };
    auto write_mom = [&](int c0, int cn) {
        for (int i = tid; i < cn * 9; i += kTileThreads) {
            const int si = i / 9, k = i - si * 9;
            a.gmom[(int64_t)c.seg_pos[sb + c0 + si] * 9 + k] = s_mom[k][si];
        }
    };

    // segments staged kSegCap at a time; each chunk's pairs are the ranges
    // of its segments in the blocks (the whole blocks when all fit)
    const bool whole = nseg <= kSegCap;
    __syncthreads();                             // br
    if (MODE & MODE_J) {
        for (int c0 = 0; c0 < max(nseg, 1); c0 += kSegCap) {
            const int cn = min(nseg - c0, kSegCap);
            if (c0 > 0) __syncthreads();
            stage(c0, cn, true);
            find_ranges(sb + c0, sb + c0 + cn, whole);
            j_tile(sb + c0, cn);
        }
        __syncthreads();
        finish_u();
        __syncthreads();
    }
    if (MODE & MODE_JT) {
        for (int c0 = 0; c0 < nseg; c0 += kSegCap) {
            const int cn = min(nseg - c0, kSegCap);
            // (MODE_J staged the last chunk and its ranges; the fused pass of
            // a tile that fits reuses them)
            if (!((MODE & MODE_J) && whole)) {
                __syncthreads();
                stage(c0, cn, false);
                find_ranges(sb + c0, sb + c0 + cn, whole);
            }
            zero_mom(cn);
            __syncthreads();
            jt_tile(sb + c0, cn);
            write_mom(c0, cn);
        }
    }
    if (MODE & MODE_J) {
        // ||J p||^2 of the tile, summed in a fixed order
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sq += __shfl_xor(sq, off, kWave);
        if (lane == 0) s_red[wid] = sq;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < NW; ++w) tot += s_red[w];
            a.jp_part[t] = tot;
        }
    }
}

template <int MODE, int DT>
__global__ void __launch_bounds__(kTileThreads, 4) k_apply_tile(ApplyBatch Bt) {
    apply_tile_body<MODE, DT>(Bt, blockIdx.x);
}

// ---- per-(Gaussian, view) sums of per-segment values ---------------------------
// The segment list grouped by (Gaussian, view) (gv_segs, ascending gv) is
// reduced with one lane per list entry and a segmented scan across each
// wave.  A group that lies inside one wave is written directly; a gv whose
// list crosses waves leaves a piece in each wave (the wave's last group, or
// its first group), and k_gv_reduce_join adds the pieces in wave order.  The
// result does not depend on scheduling.
constexpr uint32_t kNoGv = 0xFFFFFFFFu;

template <int NV>
__device__ __forceinline__ void gv_reduce_body(const CacheView& c, const float* __restrict__ src,
                                               float* __restrict__ dst, float* __restrict__ edge,
                                               uint32_t* __restrict__ edge_key, int64_t i) {
    const int64_t w = i / kWave;
    if (w >= (c.n_seg + kWave - 1) / kWave) return;   // whole waves past the list
    const int lane = __lane_id();
    const bool has = i < c.n_seg;
    float v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0f;
    uint32_t key = kNoGv;
    if (has) {   // src holds the per-segment values at their list positions
        key = c.list_gv[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = src[i * NV + k];
    }
    const uint32_t next = __shfl_down(key, 1, kWave);
    const int head = segment_head(key, lane);
    wave_segmented_scan<NV>(v, lane, head);
    const bool tail = lane == kWave - 1 || next != key;
    bool opens = false;
    if (has && tail) {
        const int64_t first = i - (lane - head);
        const bool starts = first == (int64_t)c.gv_seg_off[key];
        const bool ends = i + 1 == (int64_t)c.gv_seg_off[key + 1];
        if (starts && ends) {
#pragma unroll
            for (int k = 0; k < NV; ++k) dst[(int64_t)key * NV + k] = v[k];
        } else if (!starts) {   // continues from the previous wave: the wave's first group
#pragma unroll
            for (int k = 0; k < NV; ++k) edge[(2 * w) * NV + k] = v[k];
        } else {                // starts here and continues: the wave's last group
#pragma unroll
            for (int k = 0; k < NV; ++k) edge[(2 * w + 1) * NV + k] = v[k];
            opens = true;
        }
    }
    if (lane == kWave - 1) edge_key[w] = opens ? key : kNoGv;
}

template <int NV>
__device__ __forceinline__ void gv_reduce_join_body(const CacheView& c, const float* __restrict__ edge,
                                                    const uint32_t* __restrict__ edge_key, float* __restrict__ dst,
                                                    int64_t w) {
    const int64_t n_waves = (c.n_seg + kWave - 1) / kWave;
    if (w >= n_waves) return;
    const uint32_t key = edge_key[w];
    if (key == kNoGv) return;
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = edge[(2 * w + 1) * NV + k];
    const int64_t end = c.gv_seg_off[key + 1];
    for (int64_t u = w + 1; u * kWave < end && u < n_waves; ++u)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += edge[(2 * u) * NV + k];
#pragma unroll
    for (int k = 0; k < NV; ++k) dst[(int64_t)key * NV + k] = acc[k];
}

template <int NV>
__global__ void __launch_bounds__(kBlock) k_gv_reduce(CacheView c, const float* __restrict__ src,
                                                     float* __restrict__ dst, float* __restrict__ edge,
                                                     uint32_t* __restrict__ edge_key) {
    gv_reduce_body<NV>(c, src, dst, edge, edge_key, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

template <int NV>
__global__ void __launch_bounds__(kBlock) k_gv_reduce_join(CacheView c, const float* __restrict__ edge,
                                                          const uint32_t* __restrict__ edge_key,
                                                          float* __restrict__ dst) {
    gv_reduce_join_body<NV>(c, edge, edge_key, dst, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// the moment sums of a batch of subsets (subset = blockIdx.y)
__global__ void __launch_bounds__(kBlock) k_gv_reduce_moments(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    gv_reduce_body<9>(a.c, a.gmom, a.gvsum, a.edge, a.edge_key, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_gv_reduce_moments_join(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    gv_reduce_join_body<9>(a.c, a.edge, a.edge_key, a.gvsum, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// ---- chain: per-(Gaussian, view) moments -> parameters ---------------------------
// The adjoint of the tangent map: g_geo = sum_v L_v^T S[0:6] + Jdir_v^T S[6:9],
// g_sh[k][ch] = sum_v mask_ch Y_k S[6 + ch], with S the (Gaussian, view)'s
// moments (summed over its segments by k_gv_reduce).  Two passes, both with
// coalesced loads: one thread per (Gaussian, view) maps its moments to its
// 11 geometric (float64) and 3K SH contributions, stored per row over the
// (Gaussian, view) records; then one thread per Gaussian sums its records
// row by row (in record order).  out = scale * J^T u (+ lambda M p);
// partial dot products p . out per block.
template <int DEG>
__device__ __forceinline__ void chain_gv_body(const ApplyArgs& a, int64_t gv) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const CacheView& c = a.c;
    if (gv >= c.n_gv) return;
    const int64_t ls = c.lin_stride;
    double* __restrict__ geo_out = a.gvc;                           // [11][ls]
    float* __restrict__ sh_out = (float*)(a.gvc + 11 * ls);         // [3K][ls]
    float S9[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) S9[k] = a.gvsum[gv * 9 + k];
#pragma unroll
    for (int j = 0; j < 11; ++j) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) v += (double)c.lin[(int64_t)(kLinL + 11 * i + j) * ls + gv] * (double)S9[i];
        if (j < 3) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                v += (double)c.lin[(int64_t)(kLinJdir + 3 * ch + j) * ls + gv] * (double)S9[6 + ch];
        }
        geo_out[(int64_t)j * ls + gv] = v;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float w = c.lin[(int64_t)(kLinMask + ch) * ls + gv] * S9[6 + ch];
#pragma unroll
        for (int k = 0; k < K; ++k) sh_out[(int64_t)(3 * k + ch) * ls + gv] = c.lin[(int64_t)(kLinY + k) * ls + gv] * w;
    }
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_chain_gv(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    chain_gv_body<DEG>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Gaussian g: out = scale J^T u (+ lambda M p) over its P parameters; returns
// its share of p . out (0 past the last Gaussian)
template <int DEG>
__device__ __forceinline__ double chain_body(const ApplyBatch& Bt, const ApplyArgs& a, int64_t g) {
    const float scale = Bt.scale, lambda = Bt.lambda, diag_floor = Bt.diag_floor;
    const float* __restrict__ M = a.M;
    float* __restrict__ out = a.out;
    const bool want_pg = a.pg_part != nullptr;
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const CacheView& c = a.c;
    const int64_t ls = c.lin_stride;
    const double* __restrict__ geo_in = a.gvc;
    const float* __restrict__ sh_in = (const float*)(a.gvc + 11 * ls);
    double pg = 0.0;
    if (g < c.N) {
        const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
        const uint32_t n = e - b;
        for (int j = 0; j < P; ++j) {
            // the first four records' loads are issued together (most
            // Gaussians have at most four); the sums keep record order
            double v = 0.0;
            if (j < 11) {
                const double* row = geo_in + (int64_t)j * ls + b;
                double r[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = (uint32_t)q < n ? row[q] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) v += r[q];
                for (uint32_t q = 4; q < n; ++q) v += row[q];
            } else {
                const float* row = sh_in + (int64_t)(j - 11) * ls + b;
                float r[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = (uint32_t)q < n ? row[q] : 0.0f;
                float f = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) f += r[q];
                for (uint32_t q = 4; q < n; ++q) f += row[q];
                v = (double)f;
            }
            double val = v * scale;
            const int64_t idx = (int64_t)j * c.N + g;
            if (M) {
                const float m = M[idx];
                const float md = m > 0.0f ? fmaxf(m, diag_floor) : 0.0f;
                val += (double)lambda * (double)md * (double)a.p[idx];
            }
            out[idx] = (float)val;
            if (want_pg) pg += (double)a.p[idx] * (double)(float)val;
        }
    }
    return pg;
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_chain(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    __shared__ double s_red[kBlock / kWave];
    double pg = chain_body<DEG>(Bt, a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (a.pg_part) {
        const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) pg += __shfl_xor(pg, off, kWave);
        if (lane == 0) s_red[wid] = pg;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) tot += s_red[w];
            a.pg_part[blockIdx.x] = tot;
        }
    }
}

}  // namespace
}  // namespace lm
