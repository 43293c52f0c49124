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

// Tile pass.  One workgroup of 512 threads (8 waves) per tile.  The tile's
// pairs are stored block after block (a block is the 64 pixels of one
// raster wave), so after a block's pairs every one of its pixels has its
// complete u = J p.  A block's pairs are taken in chunks of 512 pairs (a
// window of the fill's placement rule: no piece crosses one), chunk c by
// wave c mod 8, so every piece of a chunk lies in one wave:
//   J  : the wave holds the chunk as 8 windows of 64 consecutive pairs, one
//        pair per lane (coalesced loads); per window the J rows of the
//        lanes' pairs, and the window's pieces (a contiguous lane range
//        each, distinct pixels within a piece) add into the wave's
//        per-pixel accumulators one after another with plain LDS
//        read-modify-writes; the waves' accumulators are added in wave
//        order into u;
//   J^T: the wave reads the chunk again as 64 runs of 8 pairs, one per lane
//        (a run belongs to one piece); each lane sums the 9 moments of its
//        run, one segmented scan over the wave (keyed by segment) leaves
//        each piece's sum in its last lane, which adds it into the
//        segment's moments (a segment has one piece per block, in one
//        chunk; blocks in order).
// No LDS atomics, and every sum runs in a fixed order.  The J^T read of a
// block follows its J read within microseconds (an L2 hit); each wave
// issues its first chunk of the next block before the current block's
// barriers and J^T half, so the loads overlap the other work.  A tile with
// more segments than LDS stages at once (kSegCap) runs segment chunk after
// segment chunk (J over all, then J^T).
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kSegCap = 512;
constexpr int kChunkRuns = kWave;                 // runs of a chunk (one per lane in J^T)
static_assert(kChunkRuns * kRun == kWindow, "a chunk is one placement window");
constexpr int kChunkWins = kWindow / kWave;       // 64-pair windows of a chunk (J)

// One chunk in pair order: window j's word of lane l is pair 64 j + l;
// 16-bit words two per register, pixel bytes four per register, and the
// segments of the chunk's 64 runs one per lane (run l in lane l).
template <int DT>
struct PairChunk {
    using S = Store<DT>;
    using W = typename S::word;
    static constexpr int NR = sizeof(W) == 4 ? kChunkWins : kChunkWins / 2;   // registers per plane
    uint32_t tw[NR];
    uint32_t dw[3][NR];
    uint32_t pw[kChunkWins / 4];
    uint32_t rseg;
    __device__ __forceinline__ W word(const uint32_t* p, int j) const {
        if constexpr (sizeof(W) == 4) return p[j];
        else return (W)((p[j >> 1] >> (16 * (j & 1))) & 0xFFFFu);
    }
    __device__ __forceinline__ W t(int j) const { return word(tw, j); }
    __device__ __forceinline__ W d(int ch, int j) const { return word(dw[ch], j); }
    __device__ __forceinline__ int pix(int j) const { return (int)((pw[j >> 2] >> (8 * (j & 3))) & 0xFFu); }
};

// chunk of tile-relative first pair q0 in pair order (q0 = 1 << 28 reads
// past every tile: zeros, no memory access)
template <int DT>
__device__ __forceinline__ void load_pair_chunk(const TilePlanes<DT>& P, int q0, int lane, PairChunk<DT>& L) {
    using W = typename Store<DT>::word;
    const __amdgpu_buffer_rsrc_t pr[4] = {P.t, P.d0, P.d1, P.d2};
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
        uint32_t* dst = pl == 0 ? L.tw : L.dw[pl - 1];
#pragma unroll
        for (int j = 0; j < kChunkWins; ++j) {
            const int q = q0 + kWave * j + lane;
            if constexpr (sizeof(W) == 4) {
                dst[j] = __builtin_amdgcn_raw_buffer_load_b32(pr[pl], q * 4, 0, 0);
            } else {
                const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(pr[pl], q * 2, 0, 0);
                dst[j >> 1] = (j & 1) ? (dst[j >> 1] | (h << 16)) : h;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kChunkWins; ++j) {
        const uint32_t b = __builtin_amdgcn_raw_buffer_load_b8(P.pix, q0 + kWave * j + lane, 0, 0);
        L.pw[j >> 2] = (j & 3) ? (L.pw[j >> 2] | (b << (8 * (j & 3)))) : b;
    }
    L.rseg = __builtin_amdgcn_raw_buffer_load_b32(P.seg, ((q0 / kRun) + lane) * 4, 0, 0);
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
    constexpr int kFar = 1 << 28;                // pair offset past every tile
    const CacheView& c = a.c;
    __shared__ float4 s_sg[kSegCap][4];   // mx', my', A', B' | C', o, P1, P2 | Q1, Q2, Q3, do | dc0, dc1, dc2, -
    __shared__ float s_mom[9][kSegCap];
    __shared__ float s_uw[3][NW][kBlockPix];    // per-wave J accumulators of one block, per channel
    __shared__ float4 s_ut[kMaxTilePix];        // u of the tile (weighted once complete)
    __shared__ double s_red[NW];
    __shared__ int br[kTileBlocks + 1];         // tile-relative first run of each block

    const int64_t t = gt - Bt.tile_off[bi];
    const int tid = threadIdx.x, lane = __lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int v = c.tile_view[t];
    const CamDev& cam = c.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
    const int tw_mask = c.TW - 1, tw_shift = c.tw_shift;
    const int npix = c.TW * c.TH;
    const bool blk8 = c.TW >= 8 && c.TH >= 8;
    const int bpr = c.TW >> 3;
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

    // tile pixel of pixel i of block b, and a tile pixel's index in its block
    auto blk_pixel = [&](int b, int i) -> int {
        return blk8 ? (((b / bpr) << 3) + (i >> 3)) * c.TW + ((b % bpr) << 3) + (i & 7) : b * kBlockPix + i;
    };
    auto local_of = [&](int pl) -> int { return blk8 ? (((pl >> tw_shift) & 7) << 3) | (pl & 7) : pl & (kBlockPix - 1); };
    auto pix_valid = [&](int pl) -> bool {
        return pl < npix && tx * c.TW + (pl & tw_mask) < cam.W && ty * c.TH + (pl >> tw_shift) < cam.H;
    };
    auto img_index = [&](int pl) -> int64_t {
        return 3 * cam.pix_base + (int64_t)(ty * c.TH + (pl >> tw_shift)) * cam.W + tx * c.TW + (pl & tw_mask);
    };

    for (int i = tid; i < kMaxTilePix; i += kTileThreads) s_ut[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = tid; i < 3 * NW * kBlockPix; i += kTileThreads) (&s_uw[0][0][0])[i] = 0.0f;
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
    // first pair of chunk ch of block b (kFar when the wave has no such chunk)
    auto chunk_q0 = [&](int b, int ch) -> int {
        const int r = br[b] + ch * kChunkRuns;
        return r < br[b + 1] ? r * kRun : kFar;
    };

    // J rows of one chunk (first pair q0, the block's pairs end at qe;
    // segments [s0, s0 + cn) staged) into this wave's accumulators
    auto j_chunk = [&](const PairChunk<DT>& L, int q0, int qe, int64_t s0, int cn) {
        float* u0 = s_uw[0][wid];
        float* u1 = s_uw[1][wid];
        float* u2 = s_uw[2][wid];
#pragma unroll
        for (int j = 0; j < kChunkWins; ++j) {
            const uint32_t sg = (uint32_t)__shfl((int)L.rseg, (kWave / kRun) * j + (lane >> 3), kWave);
            const int64_t sl = (int64_t)sg - s0;
            const bool live = q0 + kWave * j + lane < qe && L.t(j) != 0 && sl >= 0 && sl < cn;
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
            // within a piece)
            uint64_t todo = __ballot(live);
            while (todo) {
                const int first = __ffsll((unsigned long long)todo) - 1;
                const uint32_t sk = (uint32_t)__builtin_amdgcn_readlane((int)sg, first);
                const bool mine = live && sg == sk;
                todo &= ~__ballot(mine);
                if (mine) {
                    const int li = local_of(pl);
                    u0[li] += v0;
                    u1[li] += v1;
                    u2[li] += v2;
                }
            }
        }
    };
    // J^T moments of one chunk (lane: one run, segments [s0, s0 + cn)
    // staged): per lane the sums over its run, a segmented scan over the
    // wave, one plain addition per piece with pairs (a gap run carries the
    // next piece's segment and no pair: a group of gap runs adds nothing)
    auto jt_chunk = [&](const RunLoad<DT>& L, int64_t s0, int cn) {
        const int64_t sl = (int64_t)L.seg - s0;
        const bool in = sl >= 0 && sl < cn;
        const int key = in ? (int)sl : kNoSeg;
        float m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = 0.0f;
        bool any = false;
        {
            const int s = in ? key : 0;
            const float4 g0 = s_sg[s][0], g1 = s_sg[s][1];
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const bool live = in && L.t(k) != 0;
                any = any || live;
                const float T = S::dec_T(L.t(k));
                const bool clamped = S::clamp(L.t(k));
                const int pl = L.pix(k);
                const float dx = (float)(pl & tw_mask) - g0.x;
                const float dy = (float)(pl >> tw_shift) - g0.y;
                const float G = __builtin_amdgcn_exp2f(dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy);
                const float alpha = clamped ? 0.99f : g1.y * G;
                const float aT = live ? alpha * T : 0.0f;
                const float4 u = s_ut[pl];
                const float w = S::dec(L.d(0, k)) * u.x + S::dec(L.d(1, k)) * u.y + S::dec(L.d(2, k)) * u.z;
                const bool off = clamped || !live;
                const float aw = off ? 0.0f : alpha * w;
                const float awx = aw * dx, awy = aw * dy;
                m[0] += awx;
                m[1] += awy;
                m[2] += awx * dx;
                m[3] += awx * dy;
                m[4] += awy * dy;
                m[5] += off ? 0.0f : G * w;
                m[6] += aT * u.x;
                m[7] += aT * u.y;
                m[8] += aT * u.z;
            }
        }
        const uint64_t lives = __ballot(any);
        const int next = __shfl_down(key, 1, kWave);
        const int head = segment_head((uint32_t)key, lane);
        wave_segmented_scan<9>(m, lane, head);
        const uint64_t grp = ((2ull << lane) - 1ull) & ~((1ull << head) - 1ull);
        if (key != kNoSeg && (lane == kWave - 1 || next != key) && (lives & grp) != 0ull) {
#pragma unroll
            for (int k = 0; k < 9; ++k) s_mom[k][key] += m[k];
        }
    };
    // the block's runs in a lane: run r when it lies in block b
    auto load_run_chunk = [&](int b, int ch, RunLoad<DT>& L) {
        const int r = br[b] + ch * kChunkRuns + lane;
        P.run_if(r, L, r < br[b + 1]);
    };
    auto nchunks = [&](int b) { return (br[b + 1] - br[b] + kChunkRuns - 1) / kChunkRuns; };
    // the waves' accumulators of block b added into u (and cleared)
    auto gather_u = [&](int b) {
        if (tid < kBlockPix) {
            float4 u = make_float4(s_uw[0][0][tid], s_uw[1][0][tid], s_uw[2][0][tid], 0.0f);
            s_uw[0][0][tid] = s_uw[1][0][tid] = s_uw[2][0][tid] = 0.0f;
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                u.x += s_uw[0][w][tid];
                u.y += s_uw[1][w][tid];
                u.z += s_uw[2][w][tid];
                s_uw[0][w][tid] = s_uw[1][w][tid] = s_uw[2][w][tid] = 0.0f;
            }
            const int pl = blk_pixel(b, tid);
            if (pl < npix) {
                float4 acc = s_ut[pl];
                acc.x += u.x;
                acc.y += u.y;
                acc.z += u.z;
                s_ut[pl] = acc;
            }
        }
    };
    // u of block b complete: ||J p||^2 (sum w u^2 with residual weights),
    // the J output, and w . u for the J^T half
    double sq = 0.0;
    auto finish_u = [&](int b) {
        if (tid < kBlockPix) {
            const int pl = blk_pixel(b, tid);
            if (pl < npix) {
                const float4 u = s_ut[pl];
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
        }
    };
    auto write_mom = [&](int c0, int cn) {
        for (int i = tid; i < cn * 9; i += kTileThreads) {
            const int si = i / 9, k = i - si * 9;
            a.gmom[(int64_t)c.seg_pos[sb + c0 + si] * 9 + k] = s_mom[k][si];
        }
    };

    if (nseg <= kSegCap) {
        stage(0, nseg, (MODE & MODE_J) != 0);
        if (MODE & MODE_JT) zero_mom(nseg);
        __syncthreads();
        // first chunk of this wave in block 0 (J: pair order; J^T only: runs)
        PairChunk<DT> pj;
        RunLoad<DT> rj;
        if (MODE & MODE_J) load_pair_chunk(P, chunk_q0(0, wid), lane, pj);
        else load_run_chunk(0, wid, rj);
        for (int b = 0; b < nblk; ++b) {
            const int nch = nchunks(b);
            const int qe = br[b + 1] * kRun;
            if (MODE & MODE_J) {
                j_chunk(pj, chunk_q0(b, wid), qe, sb, nseg);
                for (int ch = wid + NW; ch < nch; ch += NW) {
                    PairChunk<DT> L;
                    const int q0 = chunk_q0(b, ch);
                    load_pair_chunk(P, q0, lane, L);
                    j_chunk(L, q0, qe, sb, nseg);
                }
                // J^T of this block reads the runs again (in cache); the
                // next block's first J chunk loads meanwhile
                if (MODE & MODE_JT) load_run_chunk(b, wid, rj);
                if (b + 1 < nblk) load_pair_chunk(P, chunk_q0(b + 1, wid), lane, pj);
                __syncthreads();
                gather_u(b);
                __syncthreads();
                finish_u(b);
                __syncthreads();
            }
            if (MODE & MODE_JT) {
                RunLoad<DT> cur = rj;
                if (!(MODE & MODE_J) && b + 1 < nblk) load_run_chunk(b + 1, wid, rj);
                jt_chunk(cur, sb, nseg);
                for (int ch = wid + NW; ch < nch; ch += NW) {
                    RunLoad<DT> L;
                    load_run_chunk(b, ch, L);
                    jt_chunk(L, sb, nseg);
                }
                // one addition per segment and block, blocks in order (the
                // fused pass orders them with the next block's J barriers)
                if (!(MODE & MODE_J)) __syncthreads();
            }
        }
        if (MODE & MODE_JT) {
            __syncthreads();
            write_mom(0, nseg);
        }
    } else {
        if (MODE & MODE_J) {
            for (int c0 = 0; c0 < nseg; c0 += kSegCap) {
                const int cn = min(nseg - c0, kSegCap);
                __syncthreads();
                stage(c0, cn, true);
                __syncthreads();
                for (int b = 0; b < nblk; ++b) {
                    const int qe = br[b + 1] * kRun;
                    for (int ch = wid; ch < nchunks(b); ch += NW) {
                        PairChunk<DT> L;
                        const int q0 = chunk_q0(b, ch);
                        load_pair_chunk(P, q0, lane, L);
                        j_chunk(L, q0, qe, sb + c0, cn);
                    }
                    __syncthreads();
                    gather_u(b);
                    __syncthreads();
                }
            }
            for (int b = 0; b < nblk; ++b) finish_u(b);
        }
        if (MODE & MODE_JT) {
            for (int c0 = 0; c0 < nseg; c0 += kSegCap) {
                const int cn = min(nseg - c0, kSegCap);
                __syncthreads();
                stage(c0, cn, false);
                zero_mom(cn);
                __syncthreads();
                for (int b = 0; b < nblk; ++b) {
                    for (int ch = wid; ch < nchunks(b); ch += NW) {
                        RunLoad<DT> L;
                        load_run_chunk(b, ch, L);
                        jt_chunk(L, sb + c0, cn);
                    }
                    __syncthreads();
                }
                write_mom(c0, cn);
            }
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
