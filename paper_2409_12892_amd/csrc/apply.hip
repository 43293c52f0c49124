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
// tangent kernel maps p to per-(Gaussian,view) power coefficients before the
// pair pass, the chain kernel maps per-(Gaussian,view) moments back to the
// parameters after it (supplement A.2 splits applyJT the same way).
//
// Pair pass: one workgroup per tile.  Every segment (the pairs of one splat
// in one tile, in pixel order) starts on a multiple of 8 pairs and is padded
// with zero words, so each aligned run of 8 pairs belongs to exactly one
// segment, named by the run -> segment table.  A lane takes one run (vector
// loads of every cache plane, the next run prefetched while the current one
// is processed), reads its segment's splat data once from LDS and
//   J  : adds each pair's colour derivative to the pixel's LDS accumulator
//        (pixel accumulators are padded by one word per 8 pixels, so the
//        8-pair stride between neighbouring lanes does not hit one bank),
//   J^T: sums the 9 moments of its 8 pairs in registers; a segmented scan over
//        the wave (keyed by segment, runs ascending across lanes) leaves one
//        LDS add per segment and wave.
// The fused J^T J pass keeps u in LDS between the two halves (every pixel's
// splats live in its own tile), so u never reaches HBM.
#include "proj_math.h"

namespace lm {
namespace {

constexpr int kThreads = 512;  // threads per tile workgroup (8 wave64)
constexpr int kChunk = 256;    // segments staged per LDS chunk
constexpr int kRun = 8;        // pairs per run (segments are padded to runs)
// pixel accumulators: padded pixel slots [0, 287), a zero slot that is never
// written (read by padding pairs in J^T) and one sink slot per lane (written
// by padding pairs in J), so the per-pair code has no branches
constexpr int kUZero = kMaxTilePix + kMaxTilePix / 8 - 1;
constexpr int kUSink = kUZero + 1;
constexpr int kUTot = kUSink + kWave;
constexpr int MODE_J = 1, MODE_JT = 2, MODE_JTJ = 3;

__device__ __forceinline__ int upad(int pl) { return pl + (pl >> 3); }

template <int DT>
struct RunLoad {
    using S = Store<DT>;
    using W = typename S::word;
    W t[kRun];
    W d[3][kRun];
    uint8_t pix[kRun];
    uint32_t seg;
    __device__ __forceinline__ void load(const CacheView& c, int64_t run) {
        const int64_t qr = run * kRun;
        seg = c.run_seg[run];
        if constexpr (sizeof(W) == 4) {
            const uint4* pt = (const uint4*)((const uint32_t*)c.pT + qr);
            uint4 a = pt[0], b = pt[1];
            t[0] = a.x; t[1] = a.y; t[2] = a.z; t[3] = a.w; t[4] = b.x; t[5] = b.y; t[6] = b.z; t[7] = b.w;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const uint4* pd = (const uint4*)((const uint32_t*)c.pD + ch * c.pair_stride + qr);
                uint4 e = pd[0], f = pd[1];
                d[ch][0] = e.x; d[ch][1] = e.y; d[ch][2] = e.z; d[ch][3] = e.w;
                d[ch][4] = f.x; d[ch][5] = f.y; d[ch][6] = f.z; d[ch][7] = f.w;
            }
        } else {
            const uint4 a = *(const uint4*)((const uint16_t*)c.pT + qr);
            const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) { t[2 * i] = (W)(wa[i] & 0xFFFF); t[2 * i + 1] = (W)(wa[i] >> 16); }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const uint4 e = *(const uint4*)((const uint16_t*)c.pD + ch * c.pair_stride + qr);
                const uint32_t we[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) { d[ch][2 * i] = (W)(we[i] & 0xFFFF); d[ch][2 * i + 1] = (W)(we[i] >> 16); }
            }
        }
        const uint2 px = *(const uint2*)(c.ppix + qr);
#pragma unroll
        for (int i = 0; i < 4; ++i) { pix[i] = (px.x >> (8 * i)) & 0xFF; pix[4 + i] = (px.y >> (8 * i)) & 0xFF; }
    }
};

// ---- tangent: p -> per-(Gaussian, view) power coefficients -------------------
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_tangent(ApplyArgs a) {
    if (a.stop && *a.stop) return;
    const CacheView& c = a.c;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
    if (b == e) return;
    double dgeo[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) dgeo[j] = (double)a.p[(int64_t)j * c.N + g];
    for (uint32_t gv = b; gv < e; ++gv) {
        const int v = (int)(c.gv_rec[gv] / c.N);
        const CamDev& cam = c.cams[v];
        ProjFwd f;
        proj_forward<DEG>(cam, a.x, c.N, g, f);
        double out[9];
        proj_tangent<DEG>(cam, f, dgeo, a.x, a.p, c.N, g, out);
#pragma unroll
        for (int k = 0; k < 9; ++k) a.dyc[(int64_t)gv * 9 + k] = (float)out[k];
    }
}

// ---- pair pass ---------------------------------------------------------------
template <int MODE, int DT>
__global__ void __launch_bounds__(kThreads) k_apply_tile(ApplyArgs a) {
    if (a.stop && *a.stop) return;
    using S = Store<DT>;
    const CacheView& c = a.c;
    __shared__ float s_u[3][kUTot];
    __shared__ float s_seg[6][kChunk];
    __shared__ float s_tan[9][kChunk];
    __shared__ float s_mom[9][kChunk];
    __shared__ double s_red[kThreads / kWave];

    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    const int v = c.tile_view[t];
    const CamDev& cam = c.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
    const int tw_mask = c.TW - 1, tw_shift = c.tw_shift;
    const int lx = tid & tw_mask, ly = tid >> tw_shift;
    const int px = tx * c.TW + lx, py = ty * c.TH + ly;
    const bool valid = tid < c.TW * c.TH && px < cam.W && py < cam.H;
    const int64_t HW = (int64_t)cam.W * cam.H;
    const int64_t ib = 3 * cam.pix_base + (int64_t)py * cam.W + px;
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    const int nseg = (int)(se - sb);
    for (int i = tid; i < kUTot; i += kThreads)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) s_u[ch][i] = 0.0f;
    __syncthreads();
    if (MODE == MODE_JT && tid < kMaxTilePix && valid) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) s_u[ch][upad(tid)] = a.uin[ib + ch * HW];
    }

    // segments [c0, c0 + cn) of the tile: splat data (and tangents) into LDS;
    // returns their runs [r0, r1) (segment offsets are multiples of kRun)
    auto stage = [&](int c0, int cn, bool tangents, int64_t& r0, int64_t& r1) {
        for (int i = tid; i < cn; i += kThreads) {
            const int64_t s = sb + c0 + i;
#pragma unroll
            for (int k = 0; k < 6; ++k) s_seg[k][i] = c.seg_f[(int64_t)k * c.seg_stride + s];
            if (tangents) {
                const int64_t gv = c.seg_gv[s];
#pragma unroll
                for (int k = 0; k < 9; ++k) s_tan[k][i] = a.dyc[gv * 9 + k];
            }
        }
        r0 = (pb + c.seg_loc[sb + c0]) / kRun;
        r1 = (c0 + cn < nseg ? pb + c.seg_loc[sb + c0 + cn] : pe) / kRun;
    };

    // ---------------- J p ----------------
    if (MODE & MODE_J) {
        for (int c0 = 0; c0 < nseg; c0 += kChunk) {
            const int cn = nseg - c0 < kChunk ? nseg - c0 : kChunk;
            int64_t r0, r1;
            __syncthreads();
            stage(c0, cn, true, r0, r1);
            __syncthreads();
            RunLoad<DT> nxt;
            if (r0 + tid < r1) nxt.load(c, r0 + tid);
            for (int64_t run = r0 + tid; run < r1; run += kThreads) {
                const RunLoad<DT> L = nxt;
                if (run + kThreads < r1) nxt.load(c, run + kThreads);
                const int s = (int)L.seg - c0;
                if ((unsigned)s >= (unsigned)cn) continue;   // never, for a consistent cache
                const float mx = s_seg[0][s], my = s_seg[1][s], A = s_seg[2][s], B = s_seg[3][s];
                const float C = s_seg[4][s], o = s_seg[5][s];
                const float P1 = s_tan[0][s], P2 = s_tan[1][s], Q1 = s_tan[2][s], Q2 = s_tan[3][s];
                const float Q3 = s_tan[4][s], dop = s_tan[5][s];
                const float dc0 = s_tan[6][s], dc1 = s_tan[7][s], dc2 = s_tan[8][s];
#pragma unroll
                for (int k = 0; k < kRun; ++k) {
                    const float T = S::dec_T(L.t[k]);
                    const bool clamped = S::clamp(L.t[k]);
                    const int pl = L.pix[k];
                    const float dx = (float)(pl & tw_mask) + 0.5f - mx;
                    const float dy = (float)(pl >> tw_shift) + 0.5f - my;
                    const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
                    const float G = __expf(power);
                    const float alpha = clamped ? 0.99f : o * G;
                    const float aT = alpha * T;
                    const float dal_f = alpha * (dx * (P1 + Q1 * dx + Q2 * dy) + dy * (P2 + Q3 * dy)) + G * dop;
                    const float dal = clamped ? 0.0f : dal_f;
                    const int ui = L.t[k] != 0 ? upad(pl) : kUSink + lane;   // padding -> sink
                    atomicAdd(&s_u[0][ui], S::dec(L.d[0][k]) * dal + aT * dc0);
                    atomicAdd(&s_u[1][ui], S::dec(L.d[1][k]) * dal + aT * dc1);
                    atomicAdd(&s_u[2][ui], S::dec(L.d[2][k]) * dal + aT * dc2);
                }
            }
        }
        __syncthreads();
        // ||J p||^2 of the tile, and u itself for the J-only product
        double sq = 0.0;
        if (tid < kMaxTilePix && valid) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float u = s_u[ch][upad(tid)];
                sq += (double)u * (double)u;
                if (MODE == MODE_J) a.uout[ib + ch * HW] = u;
            }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sq += __shfl_xor(sq, off, kWave);
        if (lane == 0) s_red[wid] = sq;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < kThreads / kWave; ++w) tot += s_red[w];
            a.jp_part[t] = tot;
        }
        if (MODE == MODE_J) return;
    }

    // ---------------- J^T u ----------------
    for (int c0 = 0; c0 < nseg; c0 += kChunk) {
        const int cn = nseg - c0 < kChunk ? nseg - c0 : kChunk;
        int64_t r0, r1;
        __syncthreads();
        stage(c0, cn, false, r0, r1);
        for (int i = tid; i < cn; i += kThreads)
#pragma unroll
            for (int k = 0; k < 9; ++k) s_mom[k][i] = 0.0f;
        __syncthreads();
        RunLoad<DT> nxt;
        if (r0 + tid < r1) nxt.load(c, r0 + tid);
        // every lane runs every round (converged for the wave scan); lanes
        // without a run carry zeros under a key of their own
        for (int64_t base = r0; base < r1; base += kThreads) {
            const int64_t run = base + tid;
            const bool has = run < r1;
            const RunLoad<DT> L = nxt;
            if (run + kThreads < r1) nxt.load(c, run + kThreads);
            int s = has ? (int)L.seg - c0 : kChunk;
            if ((unsigned)s >= (unsigned)cn) s = kChunk;    // no run, or an inconsistent cache
            float m[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) m[k] = 0.0f;
            if (s < kChunk) {
                const float mx = s_seg[0][s], my = s_seg[1][s], A = s_seg[2][s], B = s_seg[3][s];
                const float C = s_seg[4][s], o = s_seg[5][s];
#pragma unroll
                for (int k = 0; k < kRun; ++k) {
                    const float T = S::dec_T(L.t[k]);
                    const bool clamped = S::clamp(L.t[k]);
                    const int pl = L.pix[k];
                    const float dx = (float)(pl & tw_mask) + 0.5f - mx;
                    const float dy = (float)(pl >> tw_shift) + 0.5f - my;
                    const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
                    const float G = __expf(power);
                    const float alpha = clamped ? 0.99f : o * G;
                    const float aT = alpha * T;                               // 0 for padding
                    const int ui = L.t[k] != 0 ? upad(pl) : kUZero;           // padding reads u = 0
                    const float u0 = s_u[0][ui], u1 = s_u[1][ui], u2 = s_u[2][ui];
                    const float w = S::dec(L.d[0][k]) * u0 + S::dec(L.d[1][k]) * u1 + S::dec(L.d[2][k]) * u2;
                    const float aw = clamped ? 0.0f : alpha * w;
                    const float awx = aw * dx, awy = aw * dy;
                    m[0] += awx;
                    m[1] += awy;
                    m[2] += awx * dx;
                    m[3] += awx * dy;
                    m[4] += awy * dy;
                    m[5] += clamped ? 0.0f : G * w;
                    m[6] += aT * u0;
                    m[7] += aT * u1;
                    m[8] += aT * u2;
                }
            }
            // segmented inclusive scan over the wave: runs ascend with the
            // lane, so each segment is a contiguous lane range [head, tail]
            const int prev = __shfl_up(s, 1, kWave);
            const int next = __shfl_down(s, 1, kWave);
            const uint64_t heads = __ballot(lane == 0 || prev != s);
            const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
            const int head = kWave - 1 - __clzll(heads & upto);
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const float o = __shfl_up(m[k], off, kWave);
                    if (lane - off >= head) m[k] += o;
                }
            }
            if (s < kChunk && (lane == kWave - 1 || next != s)) {
#pragma unroll
                for (int k = 0; k < 9; ++k) atomicAdd(&s_mom[k][s], m[k]);
            }
        }
        __syncthreads();
        for (int i = tid; i < cn * 9; i += kThreads) {
            const int si = i / 9, k = i - si * 9;
            a.gmom[(sb + c0 + si) * 9 + k] = s_mom[k][si];
        }
    }
}

// ---- chain: per-(Gaussian, view) moments -> parameters ---------------------------
// out = scale * J^T u (+ lambda M p); partial dot products p . out per block.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_chain(ApplyArgs a, float scale, float lambda, const float* __restrict__ M,
                                                 float diag_floor, float* __restrict__ out,
                                                 double* __restrict__ pg_part) {
    if (a.stop && *a.stop) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const CacheView& c = a.c;
    __shared__ double s_red[kBlock / kWave];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < c.N;
    double pg = 0.0;
    if (live) {
        double geo[11];
#pragma unroll
        for (int j = 0; j < 11; ++j) geo[j] = 0.0;
        double gsh[3 * K];
#pragma unroll
        for (int j = 0; j < 3 * K; ++j) gsh[j] = 0.0;
        const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
        for (uint32_t gv = b; gv < e; ++gv) {
            double S9[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) S9[k] = 0.0;
            for (uint32_t i = c.gv_seg_off[gv]; i < c.gv_seg_off[gv + 1]; ++i) {
                const int64_t s = c.gv_segs[i];
#pragma unroll
                for (int k = 0; k < 9; ++k) S9[k] += (double)a.gmom[s * 9 + k];
            }
            const int v = (int)(c.gv_rec[gv] / c.N);
            const CamDev& cam = c.cams[v];
            ProjFwd f;
            proj_forward<DEG>(cam, a.x, c.N, g, f);
            double Gy[9];
            moments_to_Gy(f, S9, Gy);
            proj_adjoint<DEG>(cam, f, Gy, a.x, c.N, g, geo, gsh);
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            double val = (j < 11 ? geo[j < 11 ? j : 0] : gsh[j >= 11 ? j - 11 : 0]) * scale;
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
// D (b . a) + e dc.  Its squared norm summed over pairs needs
//   Bbb = sum (D.D) b b^T (21), Ebd = sum e b D^T (18), E2 = sum e^2 (1).
constexpr int kGram = 40;

__device__ __forceinline__ constexpr int tri6(int i, int k) { return i * 6 - (i * (i - 1)) / 2 + (k - i); }

template <int DT>
__global__ void __launch_bounds__(kBlock) k_gram_tile(CacheView c, float* __restrict__ gram) {
    using S = Store<DT>;
    using W = typename S::word;
    const int64_t t = blockIdx.x;
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    const int tw_mask = c.TW - 1, tw_shift = c.tw_shift;
    for (int64_t s = sb + wid; s < se; s += kBlock / kWave) {
        const int64_t ss = c.seg_stride;
        const float mlx = c.seg_f[s], mly = c.seg_f[ss + s];
        const float A = c.seg_f[2 * ss + s], B = c.seg_f[3 * ss + s], C = c.seg_f[4 * ss + s];
        const float o = c.seg_f[5 * ss + s];
        const int64_t q0 = pb + c.seg_loc[s];
        const int64_t q1 = (s + 1 < se) ? pb + c.seg_loc[s + 1] : pe;
        float acc[kGram];
#pragma unroll
        for (int k = 0; k < kGram; ++k) acc[k] = 0.0f;
        for (int64_t q = q0 + lane; q < q1; q += kWave) {
            const W tw = ((const W*)c.pT)[q];
            if (tw == 0) continue;                   // padding
            const float T = S::dec_T(tw);
            const bool clamped = S::clamp(tw);
            const float D0 = S::dec(((const W*)c.pD)[q]);
            const float D1 = S::dec(((const W*)c.pD)[c.pair_stride + q]);
            const float D2 = S::dec(((const W*)c.pD)[2 * c.pair_stride + q]);
            const int pl = c.ppix[q];
            const float dx = (float)(pl & tw_mask) + 0.5f - mlx, dy = (float)(pl >> tw_shift) + 0.5f - mly;
            const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
            const float G = __expf(power);
            const float alpha = clamped ? 0.99f : o * G;
            const float e = alpha * T;
            float bb[6];
            if (clamped) {
#pragma unroll
                for (int i = 0; i < 6; ++i) bb[i] = 0.0f;
            } else {
                bb[0] = alpha * dx; bb[1] = alpha * dy; bb[2] = alpha * dx * dx;
                bb[3] = alpha * dx * dy; bb[4] = alpha * dy * dy; bb[5] = G;
            }
            const float DD = D0 * D0 + D1 * D1 + D2 * D2;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int k = i; k < 6; ++k) acc[tri6(i, k)] += DD * bb[i] * bb[k];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const float eb = e * bb[i];
                acc[21 + 3 * i] += eb * D0;
                acc[22 + 3 * i] += eb * D1;
                acc[23 + 3 * i] += eb * D2;
            }
            acc[39] += e * e;
        }
#pragma unroll
        for (int k = 0; k < kGram; ++k) {
            float vsum = acc[k];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) vsum += __shfl_xor(vsum, off, kWave);
            acc[k] = vsum;
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kGram; ++k) gram[s * kGram + k] = acc[k];
        }
    }
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_diag_gauss(CacheView c, const float* __restrict__ x,
                                                      const float* __restrict__ gram, float* __restrict__ M) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    double dgeo_acc[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) dgeo_acc[j] = 0.0;
    double dsh[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) dsh[j] = 0.0;
    const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
    for (uint32_t gv = b; gv < e; ++gv) {
        double H[kGram];
#pragma unroll
        for (int k = 0; k < kGram; ++k) H[k] = 0.0;
        for (uint32_t i = c.gv_seg_off[gv]; i < c.gv_seg_off[gv + 1]; ++i) {
            const int64_t s = c.gv_segs[i];
#pragma unroll
            for (int k = 0; k < kGram; ++k) H[k] += (double)gram[s * kGram + k];
        }
        const int v = (int)(c.gv_rec[gv] / c.N);
        const CamDev& cam = c.cams[v];
        ProjFwd f;
        proj_forward<DEG>(cam, x, c.N, g, f);
#pragma unroll
        for (int j = 0; j < 11; ++j) {
            double unit[11];
#pragma unroll
            for (int i = 0; i < 11; ++i) unit[i] = i == j ? 1.0 : 0.0;
            double co[9];
            proj_tangent<DEG>(cam, f, unit, x, nullptr, c.N, g, co);
            double q = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                q += co[i] * co[i] * H[tri6(i, i)];
#pragma unroll
                for (int k = i + 1; k < 6; ++k) q += 2.0 * co[i] * co[k] * H[tri6(i, k)];
                q += 2.0 * co[i] * (H[21 + 3 * i] * co[6] + H[22 + 3 * i] * co[7] + H[23 + 3 * i] * co[8]);
            }
            q += H[39] * (co[6] * co[6] + co[7] * co[7] + co[8] * co[8]);
            dgeo_acc[j] += q;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                dsh[3 * k + ch] += f.clamp[ch] ? 0.0 : f.Y[k] * f.Y[k] * H[39];
    }
#pragma unroll
    for (int j = 0; j < P; ++j)
        M[(int64_t)j * c.N + g] = (float)(j < 11 ? dgeo_acc[j < 11 ? j : 0] : dsh[j >= 11 ? j - 11 : 0]);
}

}  // namespace

#define LM_DEG_SWITCH(deg, CALL) \
    switch (deg) {               \
        case 0: CALL(0); break;  \
        case 1: CALL(1); break;  \
        case 2: CALL(2); break;  \
        default: CALL(3); break; \
    }

hipError_t launch_tangent(const ApplyArgs& a, hipStream_t s) {
#define LM_T(D) hipLaunchKernelGGL(k_tangent<D>, dim3(grid_for(a.c.N)), dim3(kBlock), 0, s, a)
    LM_DEG_SWITCH(a.c.deg, LM_T)
#undef LM_T
    return hipGetLastError();
}

hipError_t launch_apply_tile(int mode, const ApplyArgs& a, hipStream_t s) {
    dim3 g((unsigned)a.c.n_tiles), b(kThreads);
#define LM_APPLY_CASE(MODE, DT) hipLaunchKernelGGL((k_apply_tile<MODE, DT>), g, b, 0, s, a)
    if (a.c.dtype == LM_CACHE_F32) {
        if (mode == MODE_J) LM_APPLY_CASE(MODE_J, LM_CACHE_F32);
        else if (mode == MODE_JT) LM_APPLY_CASE(MODE_JT, LM_CACHE_F32);
        else LM_APPLY_CASE(MODE_JTJ, LM_CACHE_F32);
    } else if (a.c.dtype == LM_CACHE_BF16) {
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

hipError_t launch_chain(const ApplyArgs& a, float scale, float lambda, const float* M, float diag_floor, float* out,
                        double* pg_part, hipStream_t s) {
#define LM_C(D)                                                                                                  \
    hipLaunchKernelGGL(k_chain<D>, dim3(grid_for(a.c.N)), dim3(kBlock), 0, s, a, scale, lambda, M, diag_floor, out, \
                       pg_part)
    LM_DEG_SWITCH(a.c.deg, LM_C)
#undef LM_C
    return hipGetLastError();
}

unsigned chain_blocks(int64_t N) { return grid_for(N); }

hipError_t launch_jacobi_diag(const CacheView& c, const float* x, float* gram, float* M, hipStream_t s) {
    dim3 b(kBlock);
    if (c.dtype == LM_CACHE_F32)
        hipLaunchKernelGGL((k_gram_tile<LM_CACHE_F32>), dim3((unsigned)c.n_tiles), b, 0, s, c, gram);
    else if (c.dtype == LM_CACHE_BF16)
        hipLaunchKernelGGL((k_gram_tile<LM_CACHE_BF16>), dim3((unsigned)c.n_tiles), b, 0, s, c, gram);
    else
        hipLaunchKernelGGL((k_gram_tile<LM_CACHE_F16>), dim3((unsigned)c.n_tiles), b, 0, s, c, gram);
#define LM_D(D) hipLaunchKernelGGL(k_diag_gauss<D>, dim3(grid_for(c.N)), b, 0, s, c, x, gram, M)
    LM_DEG_SWITCH(c.deg, LM_D)
#undef LM_D
    return hipGetLastError();
}

}  // namespace lm
