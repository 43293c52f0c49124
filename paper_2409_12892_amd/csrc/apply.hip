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
// Pair pass: one workgroup per tile.  Each lane takes an aligned run of 8
// consecutive pairs (vector loads of every cache plane), walks it serially
// and
//   J  : adds its colour derivative to the pixel's accumulator in LDS,
//   J^T: accumulates the 9 moments of the pair's segment in registers and
//        flushes them to the segment's LDS accumulator when the segment ends.
// The fused J^T J pass keeps u in LDS between the two halves (every pixel's
// splats live in its own tile), so u never reaches HBM.
#include "proj_math.h"

namespace lm {



namespace {

constexpr int kChunk = 256;    // segments staged per LDS chunk
constexpr int kRun = 8;        // consecutive pairs per lane
constexpr int MODE_J = 1, MODE_JT = 2, MODE_JTJ = 3;

__device__ __forceinline__ int find_seg(const uint32_t* s_loc, int cn, uint32_t local) {
    int lo = 0, hi = cn - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_loc[mid] <= local) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int DT>
struct RunLoad {
    using S = Store<DT>;
    using W = typename S::word;
    W t[kRun];
    W d[3][kRun];
    uint8_t pix[kRun];
    __device__ __forceinline__ void load(const CacheView& c, int64_t qr) {
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
        proj_forward(cam, a.x, c.N, g, c.deg, f);
        double out[9];
        proj_tangent(cam, f, dgeo, a.x, a.p, c.N, g, c.deg, out);
#pragma unroll
        for (int k = 0; k < 9; ++k) a.dyc[(int64_t)gv * 9 + k] = (float)out[k];
    }
}

// ---- pair pass ---------------------------------------------------------------
template <int MODE, int DT>
__global__ void __launch_bounds__(kBlock) k_apply_tile(ApplyArgs a) {
    if (a.stop && *a.stop) return;
    using S = Store<DT>;
    const CacheView& c = a.c;
    __shared__ float s_u[3][kMaxTilePix];
    __shared__ float s_pc[2][kMaxTilePix];
    __shared__ float s_seg[6][kChunk];
    __shared__ float s_tan[9][kChunk];
    __shared__ float s_mom[9][kChunk];
    __shared__ uint32_t s_loc[kChunk + 1];
    __shared__ double s_red[kBlock / kWave];

    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    const int v = c.tile_view[t];
    const CamDev& cam = c.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
    const int lx = tid % c.TW, ly = tid / c.TW;
    const int px = tx * c.TW + lx, py = ty * c.TH + ly;
    const bool valid = tid < c.TW * c.TH && px < cam.W && py < cam.H;
    const int64_t HW = (int64_t)cam.W * cam.H;
    const int64_t ib = 3 * cam.pix_base + (int64_t)py * cam.W + px;
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    const int nseg = (int)(se - sb);
    s_pc[0][tid] = (float)lx + 0.5f;
    s_pc[1][tid] = (float)ly + 0.5f;
    if (MODE == MODE_JT) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) s_u[ch][tid] = valid ? a.uin[ib + ch * HW] : 0.0f;
    } else {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) s_u[ch][tid] = 0.0f;
    }
    __syncthreads();

    auto stage = [&](int c0, int cn, bool tangents) {
        for (int i = tid; i < cn; i += kBlock) {
            const int64_t s = sb + c0 + i;
#pragma unroll
            for (int k = 0; k < 6; ++k) s_seg[k][i] = c.seg_f[(int64_t)k * c.seg_stride + s];
            s_loc[i] = c.seg_loc[s];
            if (tangents) {
                const int64_t gv = c.seg_gv[s];
#pragma unroll
                for (int k = 0; k < 9; ++k) s_tan[k][i] = a.dyc[gv * 9 + k];
            }
        }
        if (tid == 0) s_loc[cn] = (c0 + cn < nseg) ? c.seg_loc[sb + c0 + cn] : (uint32_t)(pe - pb);
    };

    // ---------------- J p ----------------
    if (MODE & MODE_J) {
        for (int c0 = 0; c0 < nseg; c0 += kChunk) {
            const int cn = nseg - c0 < kChunk ? nseg - c0 : kChunk;
            stage(c0, cn, true);
            __syncthreads();
            const int64_t qb = pb + s_loc[0], qe = pb + s_loc[cn];
            const int64_t q0 = qb & ~(int64_t)(kRun - 1);
            const int64_t nruns = (qe - q0 + kRun - 1) / kRun;
            for (int64_t run = tid; run < nruns; run += kBlock) {
                const int64_t qr = q0 + run * kRun;
                RunLoad<DT> L;
                L.load(c, qr);
                const int64_t qf = qr > qb ? qr : qb;
                int s = find_seg(s_loc, cn, (uint32_t)(qf - pb));
#pragma unroll
                for (int k = 0; k < kRun; ++k) {
                    const int64_t q = qr + k;
                    if (q < qb || q >= qe) continue;
                    if (q > qf && S::head(L.t[k])) ++s;
                    const float T = S::dec_T(L.t[k]);
                    const bool clamped = S::clamp(L.t[k]);
                    const int pl = L.pix[k];
                    const float dx = s_pc[0][pl] - s_seg[0][s], dy = s_pc[1][pl] - s_seg[1][s];
                    const float A = s_seg[2][s], B = s_seg[3][s], C = s_seg[4][s];
                    const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
                    const float G = __expf(power);
                    const float alpha = clamped ? 0.99f : s_seg[5][s] * G;
                    const float aT = alpha * T;
                    float dal = 0.0f;
                    if (!clamped) {
                        const float poly = dx * (s_tan[0][s] + s_tan[2][s] * dx + s_tan[3][s] * dy) +
                                           dy * (s_tan[1][s] + s_tan[4][s] * dy);
                        dal = alpha * poly + G * s_tan[5][s];
                    }
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch)
                        atomicAdd(&s_u[ch][pl], S::dec(L.d[ch][k]) * dal + aT * s_tan[6 + ch][s]);
                }
            }
            __syncthreads();
        }
        // ||J p||^2 of the tile, and u itself for the J-only product
        double sq = 0.0;
        if (valid) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float u = s_u[ch][tid];
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
            for (int w = 0; w < kBlock / kWave; ++w) tot += s_red[w];
            a.jp_part[t] = tot;
        }
        if (MODE == MODE_J) return;
    }

    // ---------------- J^T u ----------------
    for (int c0 = 0; c0 < nseg; c0 += kChunk) {
        const int cn = nseg - c0 < kChunk ? nseg - c0 : kChunk;
        __syncthreads();
        stage(c0, cn, false);
        for (int i = tid; i < cn; i += kBlock)
#pragma unroll
            for (int k = 0; k < 9; ++k) s_mom[k][i] = 0.0f;
        __syncthreads();
        const int64_t qb = pb + s_loc[0], qe = pb + s_loc[cn];
        const int64_t q0 = qb & ~(int64_t)(kRun - 1);
        const int64_t nruns = (qe - q0 + kRun - 1) / kRun;
        for (int64_t run = tid; run < nruns; run += kBlock) {
            const int64_t qr = q0 + run * kRun;
            RunLoad<DT> L;
            L.load(c, qr);
            const int64_t qf = qr > qb ? qr : qb;
            int s = find_seg(s_loc, cn, (uint32_t)(qf - pb));
            float m[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) m[k] = 0.0f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const int64_t q = qr + k;
                if (q < qb || q >= qe) continue;
                if (q > qf && S::head(L.t[k])) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) { atomicAdd(&s_mom[i][s], m[i]); m[i] = 0.0f; }
                    ++s;
                }
                any = true;
                const float T = S::dec_T(L.t[k]);
                const bool clamped = S::clamp(L.t[k]);
                const int pl = L.pix[k];
                const float dx = s_pc[0][pl] - s_seg[0][s], dy = s_pc[1][pl] - s_seg[1][s];
                const float A = s_seg[2][s], B = s_seg[3][s], C = s_seg[4][s];
                const float power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
                const float G = __expf(power);
                const float alpha = clamped ? 0.99f : s_seg[5][s] * G;
                const float aT = alpha * T;
                const float u0 = s_u[0][pl], u1 = s_u[1][pl], u2 = s_u[2][pl];
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
            if (any) {
#pragma unroll
                for (int i = 0; i < 9; ++i) atomicAdd(&s_mom[i][s], m[i]);
            }
        }
        __syncthreads();
        for (int i = tid; i < cn * 9; i += kBlock) {
            const int si = i / 9, k = i - si * 9;
            a.gmom[(sb + c0 + si) * 9 + k] = s_mom[k][si];
        }
    }
}

// ---- chain: per-(Gaussian, view) moments -> parameters ---------------------------
// out = scale * J^T u (+ lambda M p); partial dot products p . out per block.
__global__ void __launch_bounds__(kBlock) k_chain(ApplyArgs a, float scale, float lambda, const float* __restrict__ M,
                                                 float diag_floor, float* __restrict__ out,
                                                 double* __restrict__ pg_part) {
    if (a.stop && *a.stop) return;
    const CacheView& c = a.c;
    __shared__ double s_red[kBlock / kWave];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < c.N;
    double pg = 0.0;
    if (live) {
        double geo[11];
#pragma unroll
        for (int j = 0; j < 11; ++j) geo[j] = 0.0;
        double gsh[48];
        const int nsh = c.P - 11;
        for (int j = 0; j < 48; ++j) gsh[j] = 0.0;
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
            proj_forward(cam, a.x, c.N, g, c.deg, f);
            double Gy[9];
            moments_to_Gy(f, S9, Gy);
            proj_adjoint(cam, f, Gy, a.x, c.N, g, c.deg, geo, gsh);
        }
        for (int j = 0; j < c.P; ++j) {
            double val = j < 11 ? geo[j] : gsh[j - 11];
            val *= scale;
            const int64_t idx = (int64_t)j * c.N + g;
            if (M) {
                const float m = M[idx];
                const float md = m > 0.0f ? fmaxf(m, diag_floor) : 0.0f;
                val += (double)lambda * (double)md * (double)a.p[idx];
            }
            out[idx] = (float)val;
            if (pg_part) pg += (double)a.p[idx] * (double)(float)val;
        }
        (void)nsh;
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

__device__ __forceinline__ int tri6(int i, int k) { return i * 6 - (i * (i - 1)) / 2 + (k - i); }

template <int DT>
__global__ void __launch_bounds__(kBlock) k_gram_tile(CacheView c, float* __restrict__ gram) {
    using S = Store<DT>;
    using W = typename S::word;
    const int64_t t = blockIdx.x;
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
    const int v = c.tile_view[t];
    const int64_t pb = c.tile_pair_off[t], pe = c.tile_pair_off[t + 1];
    const int64_t sb = c.tile_seg_off[t], se = c.tile_seg_off[t + 1];
    (void)v;
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
            const float T = S::dec_T(tw);
            const bool clamped = S::clamp(tw);
            const float D0 = S::dec(((const W*)c.pD)[q]);
            const float D1 = S::dec(((const W*)c.pD)[c.pair_stride + q]);
            const float D2 = S::dec(((const W*)c.pD)[2 * c.pair_stride + q]);
            const int pl = c.ppix[q];
            const float dx = (float)(pl % c.TW) + 0.5f - mlx, dy = (float)(pl / c.TW) + 0.5f - mly;
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

__global__ void __launch_bounds__(kBlock) k_diag_gauss(CacheView c, const float* __restrict__ x,
                                                      const float* __restrict__ gram, float* __restrict__ M) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    double dgeo_acc[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) dgeo_acc[j] = 0.0;
    double dsh[48];
    for (int j = 0; j < 48; ++j) dsh[j] = 0.0;
    const int K = (c.deg + 1) * (c.deg + 1);
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
        proj_forward(cam, x, c.N, g, c.deg, f);
        for (int j = 0; j < 11; ++j) {
            double unit[11];
#pragma unroll
            for (int i = 0; i < 11; ++i) unit[i] = i == j ? 1.0 : 0.0;
            double co[9];
            proj_tangent(cam, f, unit, x, nullptr, c.N, g, c.deg, co);
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
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (!f.clamp[ch]) dsh[3 * k + ch] += f.Y[k] * f.Y[k] * H[39];
    }
    for (int j = 0; j < c.P; ++j) M[(int64_t)j * c.N + g] = (float)(j < 11 ? dgeo_acc[j] : dsh[j - 11]);
}

}  // namespace

hipError_t launch_tangent(const ApplyArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tangent, dim3(grid_for(a.c.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_apply_tile(int mode, const ApplyArgs& a, hipStream_t s) {
    dim3 g((unsigned)a.c.n_tiles), b(kBlock);
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
    hipLaunchKernelGGL(k_chain, dim3(grid_for(a.c.N)), dim3(kBlock), 0, s, a, scale, lambda, M, diag_floor, out,
                       pg_part);
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
    hipLaunchKernelGGL(k_diag_gauss, dim3(grid_for(c.N)), b, 0, s, c, x, gram, M);
    return hipGetLastError();
}

}  // namespace lm
