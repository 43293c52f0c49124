// Jacobian products from the gradient cache (paper section 3.3 and
// supplement A): u = J p (eq. apply-j), g = J^T u (eq. apply-jt) and
// M = diag(J^T J) (eq. diag-jtj).
//
// The Jacobian of a pixel colour with respect to the splat attributes y of
// one contributing splat (the middle factor of eq. backward-pass) is
//     dC_ch/dy = [ D_ch dalpha/dy_geo  |  alpha T e_ch ]
// with D = dC/dalpha and T read from the cache and alpha, dalpha/dy_geo
// recomputed from the staged splat (mean, conic, opacity) and the pixel.
// The splat-to-parameter factor dy/dx is applied per (Gaussian, view): the
// projection is linearised once per cache (float64, stored as float32), the
// tangent kernel maps p through it to per-(Gaussian,view) power coefficients
// before the pair pass, and the chain kernel applies its transpose to the
// per-(Gaussian,view) moments after it (supplement A.2 splits applyJT the
// same way).
//
// Pair pass: one workgroup per tile.  Every segment (the pairs of one splat
// in one tile, in pixel order) starts on a multiple of 8 pairs and is padded
// with zero words, so each aligned run of 8 pairs belongs to exactly one
// segment, named by the run -> segment table.
//   J  : a wave takes 64 consecutive pairs at a time, one per lane, and adds
//        the colour derivatives into private per-pixel LDS accumulators; the
//        pixels of one segment are distinct, so the segment pieces of the
//        window update one after another without atomics, and the waves'
//        accumulators are summed at the end.
//   J^T: a lane takes one 8-pair run (vector loads of every cache plane, the
//        next run prefetched), sums the 9 moments of its run in registers; a
//        segmented scan over the wave (keyed by segment, runs ascending
//        across lanes) leaves one LDS add per segment and wave.
// The fused J^T J pass keeps u in LDS between the two halves (every pixel's
// splats live in its own tile), so u never reaches HBM.
#include <algorithm>

#include "proj_math.h"

namespace lm {
namespace {

constexpr int kRun = 8;        // pairs per run (pieces are padded to runs)
constexpr int MODE_J = 1, MODE_JT = 2, MODE_JTJ = 3;


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
__global__ void __launch_bounds__(kBlock) k_tangent(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const CacheView& c = a.c;
    const int64_t gv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// Tile pass.  One workgroup of 512 threads per tile.  The tile's pairs are
// stored block after block (a block is the 64 pixels of one raster wave),
// so after a block's pairs every one of its pixels has its complete
// u = J p.  In the fused J^T J pass each lane loads up to kHeld<DT> runs of
// the block into registers, adds their J rows into per-wave LDS
// accumulators (ds_add; a run's eight pixels are distinct), the waves'
// accumulators are summed into u, and the J^T half takes its moments from
// the same registers: each pair is read from HBM once.  Runs past the
// register capacity are streamed in each half.  Segment moments gather in
// LDS across the tile's blocks and are written once per segment.
//   A tile with more segments than LDS stages at once (kSegCap) runs
// segment chunk after chunk: J over every chunk's runs (each block's runs
// of a chunk are found by binary search: a block lists its pieces in depth
// order) completes u for the tile, then J^T streams the runs again.
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kSegCap = 640;
template <int DT>
struct Held {
    static constexpr int R = sizeof(typename Store<DT>::word) == 4 ? 2 : 3;   // runs held per lane
};

template <int MODE, int DT>
__global__ void __launch_bounds__(kTileThreads, 4) k_apply_tile(ApplyBatch Bt) {
    int bi = 0;
    while (bi + 1 < Bt.n && (int64_t)blockIdx.x >= Bt.tile_off[bi + 1]) ++bi;
    const ApplyArgs& a = Bt.a[bi];
    if (a.stop && *a.stop) return;
    using S = Store<DT>;
    constexpr int NW = kTileWaves;
    constexpr int R = MODE == MODE_JTJ ? Held<DT>::R : 0;
    constexpr int kZero = kMaxTilePix;           // u slot that stays 0 (read by padding)
    constexpr int kNoSeg = kSegCap;              // segment key of a lane without a run
    const CacheView& c = a.c;
    __shared__ float4 s_sg[kSegCap][4];   // mx', my', A', B' | C', o, P1, P2 | Q1, Q2, Q3, do | dc0, dc1, dc2, -
    __shared__ float s_mom[9][kSegCap];
    __shared__ float4 s_uw[NW][kBlockPix];      // per-wave J accumulators of one block
    __shared__ float4 s_ut[kMaxTilePix + 1];   // u of the tile (weighted once complete)
    __shared__ double s_red[NW];

    const int64_t t = blockIdx.x - Bt.tile_off[bi];
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
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
    int brun[kTileBlocks + 1];                   // tile-relative runs of each block
    brun[0] = 0;
#pragma unroll
    for (int b = 0; b < kTileBlocks; ++b) brun[b + 1] = brun[b] + (int)(c.tile_blk[t * kTileBlocks + b] / kRun);
    const uint32_t* rseg = c.run_seg + pb / kRun;

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
    // first run in [r0, r1) whose segment is >= key (runs ascend by segment within a block)
    auto lower = [&](int r0, int r1, uint32_t key) -> int {
        while (r0 < r1) {
            const int m = (r0 + r1) >> 1;
            if (rseg[m] < key) r0 = m + 1; else r1 = m;
        }
        return r0;
    };

    for (int i = tid; i <= kMaxTilePix; i += kTileThreads) s_ut[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = tid; i < NW * kBlockPix; i += kTileThreads) (&s_uw[0][0])[i] = make_float4(0.f, 0.f, 0.f, 0.f);
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
    // staged index of a run's segment (kNoSeg: no run, or not in the chunk)
    auto staged = [&](const RunLoad<DT>& L, bool has, int64_t s0, int cn) -> int {
        const int64_t sl = (int64_t)L.seg - s0;
        return (has && sl >= 0 && sl < cn) ? (int)sl : kNoSeg;
    };

    // J rows of one run into this wave's accumulators
    auto j_run = [&](const RunLoad<DT>& L, int s) {
        if (s == kNoSeg) return;
        const float4 g0 = s_sg[s][0], g1 = s_sg[s][1], g2 = s_sg[s][2], g3 = s_sg[s][3];
        float4* up = s_uw[wid];
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            if (L.t(k) == 0) continue;                  // padding
            const float T = S::dec_T(L.t(k));
            const bool clamped = S::clamp(L.t(k));
            const int pl = L.pix(k);
            const float dx = (float)(pl & tw_mask) - g0.x;
            const float dy = (float)(pl >> tw_shift) - g0.y;
            const float G = __builtin_amdgcn_exp2f(dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy);
            const float alpha = clamped ? 0.99f : g1.y * G;
            const float aT = alpha * T;
            const float dal_f = alpha * (dx * (g1.z + g2.x * dx + g2.y * dy) + dy * (g1.w + g2.z * dy)) + G * g2.w;
            const float dal = clamped ? 0.0f : dal_f;
            const int li = local_of(pl);
            atomicAdd(&up[li].x, S::dec(L.d(0, k)) * dal + aT * g3.x);
            atomicAdd(&up[li].y, S::dec(L.d(1, k)) * dal + aT * g3.y);
            atomicAdd(&up[li].z, S::dec(L.d(2, k)) * dal + aT * g3.z);
        }
    };
    // J^T moments of one run per lane, reduced over the wave's lanes by
    // segment (runs ascend with the lane) and added into the segment sums
    auto jt_round = [&](const RunLoad<DT>& L, int s) {
        float m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = 0.0f;
        if (s != kNoSeg) {
            const float4 g0 = s_sg[s][0], g1 = s_sg[s][1];
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const float T = S::dec_T(L.t(k));
                const bool clamped = S::clamp(L.t(k));
                const int pl = L.pix(k);
                const float dx = (float)(pl & tw_mask) - g0.x;
                const float dy = (float)(pl >> tw_shift) - g0.y;
                const float G = __builtin_amdgcn_exp2f(dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy);
                const float alpha = clamped ? 0.99f : g1.y * G;
                const float aT = alpha * T;                               // 0 for padding
                const float4 u = s_ut[L.t(k) != 0 ? pl : kZero];         // padding reads u = 0
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
        const int next = __shfl_down(s, 1, kWave);
        wave_segmented_scan<9>(m, lane, segment_head((uint32_t)s, lane));
        if (s != kNoSeg && (lane == kWave - 1 || next != s)) {
#pragma unroll
            for (int k = 0; k < 9; ++k) atomicAdd(&s_mom[k][s], m[k]);
        }
    };
    // runs [r0, r1) streamed, 512 per round, the next round loading
    auto stream_j = [&](int r0, int r1, int64_t s0, int cn) {
        if (r0 >= r1) return;
        RunLoad<DT> nxt;
        P.run(r0 + tid, nxt);
        for (int base = r0; base < r1; base += kTileThreads) {
            const RunLoad<DT> L = nxt;
            const bool has = base + tid < r1;
            if (base + kTileThreads < r1) P.run(base + kTileThreads + tid, nxt);
            j_run(L, staged(L, has, s0, cn));
        }
    };
    auto stream_jt = [&](int r0, int r1, int64_t s0, int cn) {
        if (r0 >= r1) return;
        RunLoad<DT> nxt;
        P.run(r0 + tid, nxt);
        for (int base = r0; base < r1; base += kTileThreads) {
            const RunLoad<DT> L = nxt;
            const bool has = base + tid < r1;
            if (base + kTileThreads < r1) P.run(base + kTileThreads + tid, nxt);
            jt_round(L, staged(L, has, s0, cn));
        }
    };
    // the waves' accumulators of block b added into u (and cleared)
    auto gather_u = [&](int b) {
        if (tid < kBlockPix) {
            float4 u = s_uw[0][tid];
            s_uw[0][tid] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                const float4 o = s_uw[w][tid];
                s_uw[w][tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                u.x += o.x;
                u.y += o.y;
                u.z += o.z;
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
        for (int b = 0; b < nblk; ++b) {
            const int r0 = brun[b], r1 = brun[b + 1];
            if (r0 == r1) continue;
            const int rh = R > 0 ? min(r1, r0 + R * kTileThreads) : r0;   // runs held in registers
            RunLoad<DT> held[R > 0 ? R : 1];
            int hs[R > 0 ? R : 1];
            if (MODE & MODE_J) {
                // runs past the register capacity first (streamed), so that
                // the held runs and the stream's buffers are never live together
                stream_j(rh, r1, sb, nseg);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int run = r0 + k * kTileThreads + tid;
                    P.run(run, held[k]);
                    hs[k] = staged(held[k], run < rh, sb, nseg);
                }
#pragma unroll
                for (int k = 0; k < R; ++k) j_run(held[k], hs[k]);
                __syncthreads();
                gather_u(b);
                __syncthreads();
                finish_u(b);
                __syncthreads();
            }
            if (MODE & MODE_JT) {
#pragma unroll
                for (int k = 0; k < R; ++k) jt_round(held[k], hs[k]);
                stream_jt(rh, r1, sb, nseg);
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
                    const int lo = lower(brun[b], brun[b + 1], (uint32_t)(sb + c0));
                    const int hi = lower(lo, brun[b + 1], (uint32_t)(sb + c0 + cn));
                    if (lo == hi) continue;
                    stream_j(lo, hi, sb + c0, cn);
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
                    const int lo = lower(brun[b], brun[b + 1], (uint32_t)(sb + c0));
                    const int hi = lower(lo, brun[b + 1], (uint32_t)(sb + c0 + cn));
                    stream_jt(lo, hi, sb + c0, cn);
                }
                __syncthreads();
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
                                               uint32_t* __restrict__ edge_key) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
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
                                                    const uint32_t* __restrict__ edge_key, float* __restrict__ dst) {
    const int64_t n_waves = (c.n_seg + kWave - 1) / kWave;
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
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
    gv_reduce_body<NV>(c, src, dst, edge, edge_key);
}

template <int NV>
__global__ void __launch_bounds__(kBlock) k_gv_reduce_join(CacheView c, const float* __restrict__ edge,
                                                          const uint32_t* __restrict__ edge_key,
                                                          float* __restrict__ dst) {
    gv_reduce_join_body<NV>(c, edge, edge_key, dst);
}

// the moment sums of a batch of subsets (subset = blockIdx.y)
__global__ void __launch_bounds__(kBlock) k_gv_reduce_moments(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    gv_reduce_body<9>(a.c, a.gmom, a.gvsum, a.edge, a.edge_key);
}

__global__ void __launch_bounds__(kBlock) k_gv_reduce_moments_join(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    gv_reduce_join_body<9>(a.c, a.edge, a.edge_key, a.gvsum);
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
__global__ void __launch_bounds__(kBlock) k_chain_gv(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const CacheView& c = a.c;
    const int64_t gv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(kBlock) k_chain(ApplyBatch Bt) {
    const ApplyArgs& a = Bt.a[blockIdx.y];
    if (a.stop && *a.stop) return;
    const float scale = Bt.scale, lambda = Bt.lambda, diag_floor = Bt.diag_floor;
    const float* __restrict__ M = a.M;
    float* __restrict__ out = a.out;
    double* __restrict__ pg_part = a.pg_part;
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const CacheView& c = a.c;
    __shared__ double s_red[kBlock / kWave];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
            if (pg_part) pg += (double)a.p[idx] * (double)(float)val;
        }
    }
    if (pg_part) {
        const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) pg += __shfl_xor(pg, off, kWave);
        if (lane == 0) s_red[wid] = pg;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) tot += s_red[w];
            pg_part[blockIdx.x] = tot;
        }
    }
}

// ---- Jacobi diagonal via per-segment Gram moments -----------------------------------
// Per pair, with b = (alpha dx, alpha dy, alpha dx^2, alpha dx dy, alpha dy^2, G)
// (zero when alpha is clamped), e = alpha T and D = dC/dalpha, the pair's
// Jacobian row block applied to a tangent with power coefficients (a, dc) is
// D (b . a) + e dc.  Its squared norm, weighted per channel by the pixel's
// residual weights w (1 without weights), summed over pairs needs
//   Bbb = sum (D.wD) b b^T (21), Ebd = sum e b (wD)^T (18),
//   E2_ch = sum w_ch e^2 (3),
// and, for the preconditioner features, the number of pairs (1).
constexpr int kGram = kGramValues;

__device__ __forceinline__ constexpr int tri6(int i, int k) { return i * 6 - (i * (i - 1)) / 2 + (k - i); }

// One workgroup per tile.  The tile's segments are taken in chunks of
// kGramChunk with their Gram sums in LDS; for every block the chunk's runs
// (found by binary search: a block lists its pieces in depth order) are
// taken one per lane, each lane sums its run's 8 pairs, a segmented scan
// over the wave (runs ascend with the lane) leaves one LDS add per segment
// piece and wave, and the chunk's sums are written at the segments' list
// positions.
constexpr int kGramChunk = 256;

template <int DT>
__global__ void __launch_bounds__(kBlock) k_gram_tile(CacheView c, float* __restrict__ gram) {
    using S = Store<DT>;
    __shared__ float s_g[kGram][kGramChunk];
    __shared__ float s_sp[6][kGramChunk];
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, lane = __lane_id();
    const int v = c.tile_view[t];
    const CamDev& cam = c.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx0 = (int)(lt % cam.TX) * c.TW, ty0 = (int)(lt / cam.TX) * c.TH;
    const int tw_mask = c.TW - 1, tw_shift = c.tw_shift;
    const int64_t HW = (int64_t)cam.W * cam.H, ib0 = 3 * cam.pix_base;
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    const int nseg = (int)(se - sb);
    const TilePlanes<DT> P(c, pb, pe);
    const uint32_t* rseg = c.run_seg + pb / kRun;
    int brun[kTileBlocks + 1];
    brun[0] = 0;
#pragma unroll
    for (int b = 0; b < kTileBlocks; ++b) brun[b + 1] = brun[b] + (int)(c.tile_blk[t * kTileBlocks + b] / kRun);
    auto lower = [&](int r0, int r1, uint32_t key) -> int {
        while (r0 < r1) {
            const int m = (r0 + r1) >> 1;
            if (rseg[m] < key) r0 = m + 1; else r1 = m;
        }
        return r0;
    };
    for (int c0 = 0; c0 < nseg; c0 += kGramChunk) {
        const int cn = min(nseg - c0, kGramChunk);
        __syncthreads();
        for (int i = tid; i < cn; i += kBlock) {
            const int64_t sg = sb + c0 + i, ss = c.seg_stride;
#pragma unroll
            for (int k = 0; k < 6; ++k) s_sp[k][i] = c.seg_f[k * ss + sg];
#pragma unroll
            for (int k = 0; k < kGram; ++k) s_g[k][i] = 0.0f;
        }
        __syncthreads();
        for (int b = 0; b < kTileBlocks; ++b) {
            const int lo = lower(brun[b], brun[b + 1], (uint32_t)(sb + c0));
            const int hi = lower(lo, brun[b + 1], (uint32_t)(sb + c0 + cn));
            for (int base = lo; base < hi; base += kBlock) {
                const int run = base + tid;
                float acc[kGram];
#pragma unroll
                for (int k = 0; k < kGram; ++k) acc[k] = 0.0f;
                int key = kGramChunk;                 // no run
                if (run < hi) {
                    RunLoad<DT> L;
                    P.run(run, L);
                    const int64_t sl = (int64_t)L.seg - (sb + c0);
                    if (sl >= 0 && sl < cn) key = (int)sl;
                    if (key < kGramChunk) {
                        const float mlx = s_sp[0][key], mly = s_sp[1][key];
                        const float A = s_sp[2][key], B = s_sp[3][key], C = s_sp[4][key], o = s_sp[5][key];
#pragma unroll
                        for (int k = 0; k < kRun; ++k) {
                            const bool live = L.t(k) != 0;                  // padding contributes nothing
                            const float T = S::dec_T(L.t(k));
                            const bool clamped = S::clamp(L.t(k));
                            const float D0 = S::dec(L.d(0, k)), D1 = S::dec(L.d(1, k)), D2 = S::dec(L.d(2, k));
                            const int pl = L.pix(k);
                            const float dx = (float)(pl & tw_mask) + 0.5f - mlx, dy = (float)(pl >> tw_shift) + 0.5f - mly;
                            const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
                            const float G = __expf(power);
                            const float alpha = clamped ? 0.99f : o * G;
                            const float e = live ? alpha * T : 0.0f;
                            const float ag = (clamped || !live) ? 0.0f : alpha;
                            float bb[6];
                            bb[0] = ag * dx; bb[1] = ag * dy; bb[2] = ag * dx * dx;
                            bb[3] = ag * dx * dy; bb[4] = ag * dy * dy; bb[5] = (clamped || !live) ? 0.0f : G;
                            float w0 = 1.0f, w1 = 1.0f, w2 = 1.0f;
                            if (c.wres) {
                                const int gx = tx0 + (pl & tw_mask), gy = ty0 + (pl >> tw_shift);
                                if (live && gx < cam.W && gy < cam.H) {
                                    const int64_t ib = ib0 + (int64_t)gy * cam.W + gx;
                                    w0 = c.wres[ib];
                                    w1 = c.wres[ib + HW];
                                    w2 = c.wres[ib + 2 * HW];
                                }
                            }
                            const float WD0 = w0 * D0, WD1 = w1 * D1, WD2 = w2 * D2;
                            const float DD = WD0 * D0 + WD1 * D1 + WD2 * D2;
#pragma unroll
                            for (int i = 0; i < 6; ++i)
#pragma unroll
                                for (int j = i; j < 6; ++j) acc[tri6(i, j)] += DD * bb[i] * bb[j];
#pragma unroll
                            for (int i = 0; i < 6; ++i) {
                                const float eb = e * bb[i];
                                acc[21 + 3 * i] += eb * WD0;
                                acc[22 + 3 * i] += eb * WD1;
                                acc[23 + 3 * i] += eb * WD2;
                            }
                            const float ee = e * e;
                            acc[39] += w0 * ee;
                            acc[40] += w1 * ee;
                            acc[41] += w2 * ee;
                            acc[42] += live ? 1.0f : 0.0f;
                        }
                    }
                }
                const int next = __shfl_down(key, 1, kWave);
                wave_segmented_scan<kGram>(acc, lane, segment_head((uint32_t)key, lane));
                if (key < kGramChunk && (lane == kWave - 1 || next != key)) {
#pragma unroll
                    for (int k = 0; k < kGram; ++k) atomicAdd(&s_g[k][key], acc[k]);
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < cn * kGram; i += kBlock) {
            const int si = i / kGram, k = i - si * kGram;
            gram[(int64_t)c.seg_pos[sb + c0 + si] * kGram + k] = s_g[k][si];
        }
    }
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// diag(J^T J) per parameter: for each (Gaussian, view) the tangent of unit
// parameter j has power coefficients co = (L[.][j], Jdir[.][j]) and its
// squared Jacobian column norm is the quadratic form of the (Gaussian,
// view)'s Gram values; an SH coefficient (k, ch) has co = Y_k e_ch on the
// colour slots.  One thread per Gaussian.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_diag_gauss(CacheView c, const float* __restrict__ gvgram,
                                                      float* __restrict__ M) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    const int64_t ls = c.lin_stride;
    double dgeo_acc[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) dgeo_acc[j] = 0.0;
    float dsh[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) dsh[j] = 0.0f;
    const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
    for (uint32_t gv = b; gv < e; ++gv) {
        const float* H = gvgram + (int64_t)gv * kGram;
#pragma unroll
        for (int j = 0; j < 11; ++j) {
            double co[9];
#pragma unroll
            for (int i = 0; i < 6; ++i) co[i] = (double)c.lin[(int64_t)(kLinL + 11 * i + j) * ls + gv];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) co[6 + ch] = j < 3 ? (double)c.lin[(int64_t)(kLinJdir + 3 * ch + j) * ls + gv] : 0.0;
            double q = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                q += co[i] * co[i] * (double)H[tri6(i, i)];
#pragma unroll
                for (int k = i + 1; k < 6; ++k) q += 2.0 * co[i] * co[k] * (double)H[tri6(i, k)];
                q += 2.0 * co[i] * ((double)H[21 + 3 * i] * co[6] + (double)H[22 + 3 * i] * co[7] +
                                    (double)H[23 + 3 * i] * co[8]);
            }
            q += (double)H[39] * co[6] * co[6] + (double)H[40] * co[7] * co[7] + (double)H[41] * co[8] * co[8];
            dgeo_acc[j] += q;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float w = c.lin[(int64_t)(kLinMask + ch) * ls + gv] * H[39 + ch];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float y = c.lin[(int64_t)(kLinY + k) * ls + gv];
                dsh[3 * k + ch] += y * y * w;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j)
        M[(int64_t)j * c.N + g] = j < 11 ? (float)dgeo_acc[j < 11 ? j : 0] : dsh[j >= 11 ? j - 11 : 0];
}

// Number of (pixel, splat) pairs of each Gaussian over all views.
__global__ void __launch_bounds__(kBlock) k_coverage(CacheView c, const float* __restrict__ gvgram,
                                                    float* __restrict__ coverage) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    double pairs = 0.0;
    for (uint32_t gv = c.gv_first[g]; gv < c.gv_first[g + 1]; ++gv) pairs += (double)gvgram[(int64_t)gv * kGram + 42];
    coverage[g] = (float)pairs;
}


// Row j of the block B_g = J_g^T J_g of Gaussian g into r (see k_block_rows).
template <int DEG>
__device__ __forceinline__ void block_row(const CacheView& c, const float* __restrict__ gvgram, int64_t g, int j,
                                          float (&r)[11 + 3 * (DEG + 1) * (DEG + 1)]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int64_t ls = c.lin_stride;
    const bool jgeo = j < 11;
    const int jg = jgeo ? j : 0;                      // in-range index for the geometric loads
    const int jk = jgeo ? 0 : (j - 11) / 3, jch = jgeo ? -1 : (j - 11) % 3;
#pragma unroll
    for (int i = 0; i < P; ++i) r[i] = 0.0f;
    const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
    for (uint32_t gv = b; gv < e; ++gv) {
        const float* H = gvgram + (int64_t)gv * kGram;
        float co[9];
#pragma unroll
        for (int i = 0; i < 6; ++i) co[i] = jgeo ? c.lin[(int64_t)(kLinL + 11 * i + jg) * ls + gv] : 0.0f;
        const float yj = c.lin[(int64_t)(kLinY + jk) * ls + gv];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float jd = j < 3 ? c.lin[(int64_t)(kLinJdir + 3 * ch + jg) * ls + gv] : 0.0f;
            const float sh = ch == jch ? c.lin[(int64_t)(kLinMask + ch) * ls + gv] * yj : 0.0f;
            co[6 + ch] = jd + sh;
        }
        float w[9];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < 6; ++k) a += H[k < i ? tri6(k, i) : tri6(i, k)] * co[k];
            w[i] = a + H[21 + 3 * i] * co[6] + H[22 + 3 * i] * co[7] + H[23 + 3 * i] * co[8];
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float a = H[39 + ch] * co[6 + ch];
#pragma unroll
            for (int i = 0; i < 6; ++i) a += H[21 + 3 * i + ch] * co[i];
            w[6 + ch] = a;
        }
#pragma unroll
        for (int i = 0; i < 11; ++i) {
            float a = 0.0f;
#pragma unroll
            for (int m = 0; m < 6; ++m) a += c.lin[(int64_t)(kLinL + 11 * m + i) * ls + gv] * w[m];
            if (i < 3) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) a += c.lin[(int64_t)(kLinJdir + 3 * ch + i) * ls + gv] * w[6 + ch];
            }
            r[i] += a;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float wc = w[6 + ch] * c.lin[(int64_t)(kLinMask + ch) * ls + gv];
#pragma unroll
            for (int k = 0; k < K; ++k) r[11 + 3 * k + ch] += wc * c.lin[(int64_t)(kLinY + k) * ls + gv];
        }
    }
}

// Row j of the block B_k = J_k^T J_k of one Gaussian over its P parameters.
// In the 9 slots of a (Gaussian, view) (six power coefficients, three
// colours) the unit tangent of parameter j has coefficients co_j, and the
// slot Gram matrix is G = [[Bbb, Ebd], [Ebd^T, diag(E2)]], so
// B_ji = sum over views of co_j^T G co_i.  One thread per (Gaussian, row),
// rows of a Gaussian adjacent, so the view data is read once per wave.
// OUT = 0 writes the dense rows of the selected Gaussians ([n_sel][P][P];
// without a selection, of the Gaussians g0, g0 + 1, ...);
// OUT = 1 writes the preconditioner target of the row: with d = B_jj,
// D = max(d, floor) and the damped block B + lambda diag(D), the row-sum
// scaling t = log(D / (sum_i |B_ji| + lambda D)) and the observed flag d > 0.
template <int DEG, int OUT>
__global__ void __launch_bounds__(kBlock) k_block_rows(CacheView c, const float* __restrict__ gvgram,
                                                      const int64_t* __restrict__ sel, int64_t g0, int64_t n_rows,
                                                      float lam, float floor_, float* __restrict__ o0,
                                                      float* __restrict__ o1) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows) return;
    const int64_t s = t / P;
    const int j = (int)(t - s * P);
    const int64_t g = sel ? sel[s] : g0 + s;
    float r[P];
    block_row<DEG>(c, gvgram, g, j, r);
    if (OUT == 0) {
        float* row = o0 + (s * P + j) * P;
#pragma unroll
        for (int i = 0; i < P; ++i) row[i] = r[i];
    } else {
        float d = 0.0f, sum = 0.0f;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            d = i == j ? r[i] : d;
            sum += fabsf(r[i]);
        }
        const bool obs = d > 0.0f;
        const float D = fmaxf(d, floor_);
        o0[(int64_t)j * c.N + g] = obs ? logf(D / (sum + lam * D)) : 0.0f;
        o1[(int64_t)j * c.N + g] = obs ? 1.0f : 0.0f;
    }
}

// Block-Jacobi factors.  Per Gaussian the damped block
// A = B + lambda diag(max(d, floor)) of its own parameters (d = diag(B); a
// parameter with d = 0 keeps a unit diagonal and no coupling) is factored
// A = L L^T in registers: one wave per Gaussian, lane i computes row i of B
// (block_row) and owns row i of the factor; each step broadcasts the pivot
// and the new column with lane reads.  A non-positive pivot falls back to
// the damped diagonal (Jacobi on this Gaussian).  L is stored packed lower,
// element t = i (i + 1) / 2 + j with 1 / L_ii on the diagonal, in tiles of
// 64 Gaussians, L[g / 64][t][g % 64]; the 8 Gaussians of a workgroup are
// consecutive, so their stores to an element fill a 32-byte sector together.
constexpr int kBjWaves = 8;

template <int DEG>
__global__ void __launch_bounds__(kBjWaves * kWave) k_bj_factor(CacheView c, const float* __restrict__ gvgram,
                                                                float lam, float floor_, float* __restrict__ L,
                                                                uint32_t* __restrict__ n_fallback) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int lane = __lane_id();
    const int64_t g = (int64_t)blockIdx.x * kBjWaves + threadIdx.x / kWave;
    if (g >= c.N) return;                              // whole waves
    const int64_t N = c.N;
    float a[P];
    block_row<DEG>(c, gvgram, g, lane < P ? lane : P - 1, a);
    float d = 0.0f;
#pragma unroll
    for (int i = 0; i < P; ++i) d = i == lane ? a[i] : d;
    const uint64_t obs = __ballot(lane < P && d > 0.0f);
    const bool mine = (obs >> lane) & 1ull;
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!mine || !((obs >> i) & 1ull)) a[i] = 0.0f;
    const float dd = mine ? d + lam * fmaxf(d, floor_) : 1.0f;
#pragma unroll
    for (int i = 0; i < P; ++i) a[i] = i == lane ? dd : a[i];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const float akk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[k]), k));
        ok = ok && akk > 0.0f && akk < INFINITY;
        const float lkk = sqrtf(fmaxf(akk, 1e-30f));
        const float inv = 1.0f / lkk;
        a[k] = lane == k ? lkk : (lane > k ? a[k] * inv : a[k]);
#pragma unroll
        for (int j = k + 1; j < P; ++j) {
            const float ljk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[k]), j));
            if (lane >= j) a[j] -= a[k] * ljk;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane < P) {
        constexpr int T = P * (P + 1) / 2;
        float* Lrow = L + ((g >> 6) * (int64_t)T + lane * (lane + 1) / 2) * 64 + (g & 63);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (j > lane) continue;
            float v;
            if (j == lane) v = ok ? 1.0f / a[j] : 1.0f / sqrtf(dd);
            else v = ok ? a[j] : 0.0f;
            Lrow[j * 64] = v;
        }
    }
    if (!ok && lane == 0) atomicAdd(n_fallback, 1u);
}

// Shrinkage of the targets towards their per-parameter mean over the
// observed Gaussians: t' = mu_j + beta (t - mu_j).  Block partials over a
// fixed number of blocks per parameter, summed in order by one workgroup
// per parameter (deterministic).
constexpr int kShrinkBlocks = 1024;

__global__ void __launch_bounds__(kBlock) k_target_partials(const float* __restrict__ t, const float* __restrict__ m,
                                                           int64_t N, double* __restrict__ part) {
    const int j = blockIdx.y;
    double a = 0.0, n = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < N; g += (int64_t)gridDim.x * kBlock) {
        const float mk = m[(int64_t)j * N + g];
        a += mk != 0.0f ? (double)t[(int64_t)j * N + g] : 0.0;
        n += mk != 0.0f ? 1.0 : 0.0;
    }
    __shared__ double sh[2][kBlock / kWave];
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, kWave);
        n += __shfl_xor(n, off, kWave);
    }
    if (lane == 0) {
        sh[0][wid] = a;
        sh[1][wid] = n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sn = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            sa += sh[0][w];
            sn += sh[1][w];
        }
        double* o = part + ((int64_t)j * gridDim.x + blockIdx.x) * 2;
        o[0] = sa;
        o[1] = sn;
    }
}

__global__ void __launch_bounds__(kBlock) k_target_mean(const double* __restrict__ part, int nb,
                                                       double* __restrict__ mean) {
    const int j = blockIdx.x;
    __shared__ double sa[kBlock], sn[kBlock];
    double a = 0.0, n = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        a += part[((int64_t)j * nb + b) * 2];
        n += part[((int64_t)j * nb + b) * 2 + 1];
    }
    sa[threadIdx.x] = a;
    sn[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tn = 0.0;
        for (int k = 0; k < kBlock; ++k) {
            ta += sa[k];
            tn += sn[k];
        }
        mean[j] = tn > 0.0 ? ta / tn : 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) k_target_shrink(float* __restrict__ t, const float* __restrict__ m,
                                                         int64_t N, const double* __restrict__ mean, float beta) {
    const int j = blockIdx.y;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= N) return;
    const int64_t i = (int64_t)j * N + g;
    const double mu = mean[j];
    t[i] = m[i] != 0.0f ? (float)(mu + (double)beta * ((double)t[i] - mu)) : 0.0f;
}

// ---- preconditioner features ----------------------------------------------
// Eight per-Gaussian features: the log of the mean Jacobi diagonal over the
// parameter groups (mean, log-scale, quaternion, opacity, SH) and
// log(1 + pair count), each centred on its mean over the observed Gaussians
// (those with a non-zero diagonal) where it is finite; the opacity
// sigmoid(logit) and the mean log-scale.  Unobserved Gaussians get zeros.
constexpr int kFeatRef = 6;   // centred features

__device__ __forceinline__ bool feat_observed(const float* M, int64_t N, int P, int64_t g) {
    float sum = 0.0f;
    for (int j = 0; j < P; ++j) sum += M[(int64_t)j * N + g];
    return sum > 0.0f;
}

__global__ void __launch_bounds__(kBlock) k_feat_raw(const float* __restrict__ M, const float* __restrict__ cov,
                                                    const float* __restrict__ x, int64_t N, int P,
                                                    float* __restrict__ feat, double* __restrict__ part) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[2 * kFeatRef];
#pragma unroll
    for (int k = 0; k < 2 * kFeatRef; ++k) v[k] = 0.0;
    if (g < N) {
        const bool obs = feat_observed(M, N, P, g);
        const int lo[5] = {0, 3, 6, 10, 11}, hi[5] = {3, 6, 10, 11, P};
        float f[kFeatRef];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            float m = 0.0f;
            for (int j = lo[q]; j < hi[q]; ++j) m += M[(int64_t)j * N + g];
            f[q] = logf(m / (float)(hi[q] - lo[q]));
        }
        f[5] = log1pf(cov[g]);
#pragma unroll
        for (int q = 0; q < kFeatRef; ++q) {
            const bool ok = obs && isfinite(f[q]);
            feat[(int64_t)q * N + g] = f[q];           // centred (or zeroed) by k_feat_centre
            v[q] = ok ? (double)f[q] : 0.0;
            v[kFeatRef + q] = ok ? 1.0 : 0.0;
        }
        const float om = x[(int64_t)10 * N + g];
        feat[(int64_t)6 * N + g] = obs ? 1.0f / (1.0f + expf(-om)) : 0.0f;
        feat[(int64_t)7 * N + g] =
            obs ? (x[(int64_t)3 * N + g] + x[(int64_t)4 * N + g] + x[(int64_t)5 * N + g]) / 3.0f : 0.0f;
    }
    __shared__ double sh[2 * kFeatRef][kBlock / kWave];
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 2 * kFeatRef; ++k) {
        double a = v[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
        if (lane == 0) sh[k][wid] = a;
    }
    __syncthreads();
    if (threadIdx.x < 2 * kFeatRef) {
        double a = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) a += sh[threadIdx.x][w];
        part[(int64_t)blockIdx.x * (2 * kFeatRef) + threadIdx.x] = a;
    }
}

// One workgroup: sums the block partials in a fixed order into the centres.
__global__ void __launch_bounds__(kBlock) k_feat_ref(const double* __restrict__ part, int64_t n_part,
                                                    double* __restrict__ ref) {
    __shared__ double sh[2 * kFeatRef][kBlock];
    double v[2 * kFeatRef];
#pragma unroll
    for (int k = 0; k < 2 * kFeatRef; ++k) v[k] = 0.0;
    for (int64_t b = threadIdx.x; b < n_part; b += kBlock)
#pragma unroll
        for (int k = 0; k < 2 * kFeatRef; ++k) v[k] += part[b * (2 * kFeatRef) + k];
#pragma unroll
    for (int k = 0; k < 2 * kFeatRef; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    if (threadIdx.x < kFeatRef) {
        double a = 0.0, n = 0.0;
        for (int w = 0; w < kBlock; ++w) {
            a += sh[threadIdx.x][w];
            n += sh[kFeatRef + threadIdx.x][w];
        }
        ref[threadIdx.x] = n > 0.0 ? a / n : 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) k_feat_centre(const float* __restrict__ M, int64_t N, int P,
                                                       const double* __restrict__ ref, float* __restrict__ feat) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const bool obs = feat_observed(M, N, P, g);
#pragma unroll
    for (int q = 0; q < kFeatRef; ++q) {
        float* f = feat + (int64_t)q * N + g;
        const float raw = *f;
        *f = obs && isfinite(raw) ? (float)((double)raw - ref[q]) : 0.0f;
    }
}

}  // namespace

#define LM_DEG_SWITCH(deg, CALL) \
    switch (deg) {               \
        case 0: CALL(0); break;  \
        case 1: CALL(1); break;  \
        case 2: CALL(2); break;  \
        default: CALL(3); break; \
    }

hipError_t launch_linearize(const CacheView& c, const float* x, float* lin, hipStream_t s) {
    if (c.n_gv == 0) return hipSuccess;
#define LM_L(D) hipLaunchKernelGGL(k_linearize<D>, dim3(grid_for(c.n_gv)), dim3(kBlock), 0, s, c, x, lin)
    LM_DEG_SWITCH(c.deg, LM_L)
#undef LM_L
    return hipGetLastError();
}

static int64_t batch_max(const ApplyBatch& B, int64_t (*f)(const ApplyArgs&)) {
    int64_t m = 0;
    for (int i = 0; i < B.n; ++i) m = std::max(m, f(B.a[i]));
    return m;
}

hipError_t launch_tangent(const ApplyBatch& B, hipStream_t s) {
    const int64_t n = batch_max(B, [](const ApplyArgs& a) { return a.c.n_gv; });
    if (n == 0) return hipSuccess;
    const dim3 g(grid_for(n), (unsigned)B.n);
#define LM_T(D) hipLaunchKernelGGL(k_tangent<D>, g, dim3(kBlock), 0, s, B)
    LM_DEG_SWITCH(B.a[0].c.deg, LM_T)
#undef LM_T
    return hipGetLastError();
}

hipError_t launch_apply_tile(int mode, const ApplyBatch& B, hipStream_t s) {
    const int64_t nt = B.tile_off[B.n];
    if (nt == 0) return hipSuccess;
    dim3 g((unsigned)nt), b(kTileThreads);
#define LM_APPLY_CASE(MODE, DT) hipLaunchKernelGGL((k_apply_tile<MODE, DT>), g, b, 0, s, B)
    const int dtype = B.a[0].c.dtype;
    if (dtype == LM_CACHE_F32) {
        if (mode == MODE_J) LM_APPLY_CASE(MODE_J, LM_CACHE_F32);
        else if (mode == MODE_JT) LM_APPLY_CASE(MODE_JT, LM_CACHE_F32);
        else LM_APPLY_CASE(MODE_JTJ, LM_CACHE_F32);
    } else if (dtype == LM_CACHE_BF16) {
        if (mode == MODE_J) LM_APPLY_CASE(MODE_J, LM_CACHE_BF16);
        else if (mode == MODE_JT) LM_APPLY_CASE(MODE_JT, LM_CACHE_BF16);
        else LM_APPLY_CASE(MODE_JTJ, LM_CACHE_BF16);
    } else {
        if (mode == MODE_J) LM_APPLY_CASE(MODE_J, LM_CACHE_F16);
        else if (mode == MODE_JT) LM_APPLY_CASE(MODE_JT, LM_CACHE_F16);
        else LM_APPLY_CASE(MODE_JTJ, LM_CACHE_F16);
    }
#undef LM_APPLY_CASE
    return hipGetLastError();
}

hipError_t launch_chain(const ApplyBatch& B, hipStream_t s) {
    const int64_t ngv = batch_max(B, [](const ApplyArgs& a) { return a.c.n_gv; });
    if (ngv > 0) {
        const dim3 gg(grid_for(ngv), (unsigned)B.n);
#define LM_CG(D) hipLaunchKernelGGL(k_chain_gv<D>, gg, dim3(kBlock), 0, s, B)
        LM_DEG_SWITCH(B.a[0].c.deg, LM_CG)
#undef LM_CG
    }
    const dim3 g(chain_blocks(B.a[0].c.N), (unsigned)B.n);
#define LM_C(D) hipLaunchKernelGGL(k_chain<D>, g, dim3(kBlock), 0, s, B)
    LM_DEG_SWITCH(B.a[0].c.deg, LM_C)
#undef LM_C
    return hipGetLastError();
}

unsigned chain_blocks(int64_t N) { return grid_for(N); }

int64_t gv_reduce_waves(int64_t n_seg) { return (n_seg + kWave - 1) / kWave; }

template <int NV>
hipError_t gv_reduce(const CacheView& c, const float* src, float* dst, float* edge, uint32_t* edge_key,
                     hipStream_t s) {
    if (c.n_seg == 0) return hipSuccess;
    const int64_t nw = gv_reduce_waves(c.n_seg);
    hipLaunchKernelGGL(k_gv_reduce<NV>, dim3(grid_for(nw * kWave)), dim3(kBlock), 0, s, c, src, dst, edge, edge_key);
    hipLaunchKernelGGL(k_gv_reduce_join<NV>, dim3(grid_for(nw)), dim3(kBlock), 0, s, c, edge, edge_key, dst);
    return hipGetLastError();
}

hipError_t launch_gv_reduce_moments(const ApplyBatch& B, hipStream_t s) {
    const int64_t ns = batch_max(B, [](const ApplyArgs& a) { return a.c.n_seg; });
    if (ns == 0) return hipSuccess;
    const int64_t nw = gv_reduce_waves(ns);
    hipLaunchKernelGGL(k_gv_reduce_moments, dim3(grid_for(nw * kWave), (unsigned)B.n), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_gv_reduce_moments_join, dim3(grid_for(nw), (unsigned)B.n), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_block_rows(const CacheView& c, const float* gvgram, const int64_t* sel, int64_t n_sel, int out,
                             float lam, float floor_, float* o0, float* o1, hipStream_t s, int64_t g0) {
    const int64_t n_rows = (sel ? n_sel : (n_sel > 0 ? n_sel : c.N - g0)) * c.P;
    if (n_rows <= 0) return hipSuccess;
    const dim3 g(grid_for(n_rows)), b(kBlock);
#define LM_B(D)                                                                                                     \
    if (out == 0) hipLaunchKernelGGL((k_block_rows<D, 0>), g, b, 0, s, c, gvgram, sel, g0, n_rows, lam, floor_, o0, \
                                     o1);                                                                           \
    else hipLaunchKernelGGL((k_block_rows<D, 1>), g, b, 0, s, c, gvgram, sel, g0, n_rows, lam, floor_, o0, o1)
    LM_DEG_SWITCH(c.deg, LM_B)
#undef LM_B
    return hipGetLastError();
}

hipError_t launch_bj_factor(const CacheView& c, const float* gvgram, float lam, float floor_, float* L,
                            uint32_t* n_fallback, hipStream_t s) {
    if (c.N == 0) return hipSuccess;
    const dim3 g((unsigned)((c.N + kBjWaves - 1) / kBjWaves)), b(kBjWaves * kWave);
    switch (c.deg) {
        case 0: hipLaunchKernelGGL(k_bj_factor<0>, g, b, 0, s, c, gvgram, lam, floor_, L, n_fallback); break;
        case 1: hipLaunchKernelGGL(k_bj_factor<1>, g, b, 0, s, c, gvgram, lam, floor_, L, n_fallback); break;
        case 2: hipLaunchKernelGGL(k_bj_factor<2>, g, b, 0, s, c, gvgram, lam, floor_, L, n_fallback); break;
        default: hipLaunchKernelGGL(k_bj_factor<3>, g, b, 0, s, c, gvgram, lam, floor_, L, n_fallback); break;
    }
    return hipGetLastError();
}

int64_t shrink_scratch_doubles(int P) { return (int64_t)P * (2 * kShrinkBlocks + 1); }

hipError_t launch_target_shrink(float* t, const float* mask, int64_t N, int P, float beta, double* scratch,
                                hipStream_t s) {
    if (N == 0 || P == 0) return hipSuccess;
    const int nb = (int)std::min<int64_t>(grid_for(N), kShrinkBlocks);
    double* mean = scratch + (int64_t)P * 2 * nb;
    hipLaunchKernelGGL(k_target_partials, dim3(nb, P), dim3(kBlock), 0, s, t, mask, N, scratch);
    hipLaunchKernelGGL(k_target_mean, dim3(P), dim3(kBlock), 0, s, scratch, nb, mean);
    hipLaunchKernelGGL(k_target_shrink, dim3(grid_for(N), P), dim3(kBlock), 0, s, t, mask, N, mean, beta);
    return hipGetLastError();
}

int64_t feature_parts(int64_t N) { return grid_for(N); }

hipError_t launch_precond_features(const float* M, const float* coverage, const float* x, int64_t N, int P,
                                   float* feat, double* part, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int64_t nb = feature_parts(N);
    double* ref = part + nb * (2 * kFeatRef);
    hipLaunchKernelGGL(k_feat_raw, dim3((unsigned)nb), dim3(kBlock), 0, s, M, coverage, x, N, P, feat, part);
    hipLaunchKernelGGL(k_feat_ref, dim3(1), dim3(kBlock), 0, s, part, nb, ref);
    hipLaunchKernelGGL(k_feat_centre, dim3((unsigned)nb), dim3(kBlock), 0, s, M, N, P, ref, feat);
    return hipGetLastError();
}

hipError_t launch_gram(const CacheView& c, float* gram, float* gvgram, float* edge, uint32_t* edge_key,
                       hipStream_t s) {
    if (c.n_tiles > 0 && c.n_seg > 0) {
        const dim3 g((unsigned)c.n_tiles), b(kBlock);
        if (c.dtype == LM_CACHE_F32) hipLaunchKernelGGL((k_gram_tile<LM_CACHE_F32>), g, b, 0, s, c, gram);
        else if (c.dtype == LM_CACHE_BF16) hipLaunchKernelGGL((k_gram_tile<LM_CACHE_BF16>), g, b, 0, s, c, gram);
        else hipLaunchKernelGGL((k_gram_tile<LM_CACHE_F16>), g, b, 0, s, c, gram);
    }
    return gv_reduce<kGram>(c, gram, gvgram, edge, edge_key, s);
}

hipError_t launch_coverage(const CacheView& c, const float* gvgram, float* coverage, hipStream_t s) {
    hipLaunchKernelGGL(k_coverage, dim3(grid_for(c.N)), dim3(kBlock), 0, s, c, gvgram, coverage);
    return hipGetLastError();
}

hipError_t launch_jacobi_diag(const CacheView& c, const float* gvgram, float* M, hipStream_t s) {
    dim3 b(kBlock);
#define LM_D(D) hipLaunchKernelGGL(k_diag_gauss<D>, dim3(grid_for(c.N)), b, 0, s, c, gvgram, M)
    LM_DEG_SWITCH(c.deg, LM_D)
#undef LM_D
    return hipGetLastError();
}

}  // namespace lm
