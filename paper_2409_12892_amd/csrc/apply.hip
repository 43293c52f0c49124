// Jacobian products from the gradient cache (paper section 3.3 and
// supplement A): the kernels of products.h, the Jacobi diagonal
// (eq. diag-jtj) from per-segment Gram values, the per-Gaussian blocks,
// targets and features of the preconditioners, and their launchers.
#include "products.h"

namespace lm {
namespace {

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
// (a lower-bound search by one wave per block: a block lists its pieces in
// depth order) are
// taken one per lane, each lane sums its run's 8 pairs, a segmented scan
// over the wave (runs ascend with the lane) leaves one LDS add per segment
// piece and wave, and the chunk's sums are written at the segments' list
// positions.
constexpr int kGramChunk = 256;

template <int DT>
__global__ void __launch_bounds__(kBlock, 3) k_gram_tile(CacheView c, float* __restrict__ gram) {
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
    __shared__ int s_lohi[kTileBlocks][2];
    int brun[kTileBlocks + 1];
    brun[0] = 0;
#pragma unroll
    for (int b = 0; b < kTileBlocks; ++b) brun[b + 1] = brun[b] + (int)(c.tile_blk[t * kTileBlocks + b] / kRun);
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
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
        // the chunk's runs in each block (wave b searches block b; kBlock
        // holds one wave per block)
        static_assert(kBlock / kWave == kTileBlocks, "one wave per block");
        {
            int bb = 0;
#pragma unroll
            for (int k = 1; k < kTileBlocks; ++k) bb = wid == k ? k : bb;
            int lo = brun[0], hi = brun[1];
#pragma unroll
            for (int k = 1; k < kTileBlocks; ++k)
                if (bb == k) {
                    lo = brun[k];
                    hi = brun[k + 1];
                }
            const int rl = run_lower_bound(P.seg, lo, hi, (uint32_t)(sb + c0), lane);
            const int rh = run_lower_bound(P.seg, rl, hi, (uint32_t)(sb + c0 + cn), lane);
            if (lane == 0) {
                s_lohi[bb][0] = rl;
                s_lohi[bb][1] = rh;
            }
        }
        __syncthreads();
        for (int b = 0; b < kTileBlocks; ++b) {
            const int lo = s_lohi[b][0];
            const int hi = s_lohi[b][1];
            // rounds start on a window of the block (no piece is split
            // between waves; runs before lo belong to earlier chunks), and a
            // barrier ends each block: one addition per segment and block
            if (b > 0) __syncthreads();
            // the next round's run loads while this round's is summed
            const int start = brun[b] + ((lo - brun[b]) & ~(kWinRuns - 1));
            RunLoad<DT> nx;
            if (start < hi) P.run_if(start + tid, nx, start + tid < hi);
            for (int base = start; base < hi; base += kBlock) {
                const RunLoad<DT> L = nx;
                if (base + kBlock < hi) P.run_if(base + kBlock + tid, nx, base + kBlock + tid < hi);
                float acc[kGram];
#pragma unroll
                for (int k = 0; k < kGram; ++k) acc[k] = 0.0f;
                int key = kGramChunk;                 // no run
                {
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
                wave_piece_scan<kGram>(acc, lane, segment_head((uint32_t)key, lane));
                // one piece per segment and block, summed by one wave: a
                // plain addition by the piece's last lane (a group of gap runs
                // carries the next window's piece's segment and no pair: it
                // adds nothing, so no two lanes add to a segment at once)
                if (key < kGramChunk && (lane == kWave - 1 || next != key) && acc[kGram - 1] != 0.0f) {
#pragma unroll
                    for (int k = 0; k < kGram; ++k) s_g[k][key] += acc[k];
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
// colour slots.  The geometric forms (float64) are evaluated with one thread
// per (Gaussian, view) into geo[j][gv]; one thread per Gaussian then sums
// them over its views, in view order, and forms the SH entries.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_diag_geo_gv(CacheView c, const float* __restrict__ gvgram,
                                                       double* __restrict__ geo) {
    const int64_t gv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gv >= c.n_gv) return;
    const int64_t ls = c.lin_stride;
    const float* H = gvgram + gv * kGram;
    double h[kGram - 1];
#pragma unroll
    for (int k = 0; k < kGram - 1; ++k) h[k] = (double)H[k];
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
            q += co[i] * co[i] * h[tri6(i, i)];
#pragma unroll
            for (int k = i + 1; k < 6; ++k) q += 2.0 * co[i] * co[k] * h[tri6(i, k)];
            q += 2.0 * co[i] * (h[21 + 3 * i] * co[6] + h[22 + 3 * i] * co[7] + h[23 + 3 * i] * co[8]);
        }
        q += h[39] * co[6] * co[6] + h[40] * co[7] * co[7] + h[41] * co[8] * co[8];
        geo[(int64_t)j * ls + gv] = q;
    }
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_diag_gauss(CacheView c, const float* __restrict__ gvgram,
                                                      const double* __restrict__ geo, float* __restrict__ M) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.N) return;
    const int64_t ls = c.lin_stride;
    const uint32_t b = c.gv_first[g], e = c.gv_first[g + 1];
#pragma unroll
    for (int j = 0; j < 11; ++j) {
        double acc = 0.0;
        for (uint32_t gv = b; gv < e; ++gv) acc += geo[(int64_t)j * ls + gv];
        M[(int64_t)j * c.N + g] = (float)acc;
    }
    float dsh[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) dsh[j] = 0.0f;
    for (uint32_t gv = b; gv < e; ++gv) {
        const float* H = gvgram + (int64_t)gv * kGram;
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
    for (int j = 0; j < 3 * K; ++j) M[(int64_t)(11 + j) * c.N + g] = dsh[j];
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


// Row j of the block B_g = J_g^T J_g of Gaussian g into r (see k_block_rows),
// the views' terms summed in the precision of R.
template <int DEG, class R>
__device__ __forceinline__ void block_row(const CacheView& c, const float* __restrict__ gvgram, int64_t g, int j,
                                          R (&r)[11 + 3 * (DEG + 1) * (DEG + 1)]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int P = 11 + 3 * K;
    const int64_t ls = c.lin_stride;
    const bool jgeo = j < 11;
    const int jg = jgeo ? j : 0;                      // in-range index for the geometric loads
    const int jk = jgeo ? 0 : (j - 11) / 3, jch = jgeo ? -1 : (j - 11) % 3;
#pragma unroll
    for (int i = 0; i < P; ++i) r[i] = R(0);
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
            r[i] += R(a);
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float wc = w[6 + ch] * c.lin[(int64_t)(kLinMask + ch) * ls + gv];
#pragma unroll
            for (int k = 0; k < K; ++k) r[11 + 3 * k + ch] += R(wc * c.lin[(int64_t)(kLinY + k) * ls + gv]);
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
// OUT = 1 writes the preconditioner target of the row (relative to the
// Jacobi inverse 1/D), the row summed over views in float64: with d = B_jj,
// D = max(d, floor) and the damped block A = B + lambda diag(D), the row-sum
// scaling that bounds the Gershgorin disc of the row,
// t = log(D / sum_i |A_ji|), and the observed flag d > 0.
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
    if constexpr (OUT == 0) {
        float r[P];
        block_row<DEG>(c, gvgram, g, j, r);
        float* row = o0 + (s * P + j) * P;
#pragma unroll
        for (int i = 0; i < P; ++i) row[i] = r[i];
    } else {
        double r[P];
        block_row<DEG>(c, gvgram, g, j, r);
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) d = i == j ? r[i] : d;
        const bool obs = d > 0.0;
        const double D = fmax(d, (double)floor_);
        const double ajj = d + (double)lam * D;
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) sum += fabs(i == j ? ajj : r[i]);
        o0[(int64_t)j * c.N + g] = obs ? (float)log(D / sum) : 0.0f;
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
    if (B.a[0].c.thin_k > 0) return launch_thin_tile(mode, B, s);
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
    if (c.thin_k > 0) {
        hipError_t e = launch_thin_gram(c, gram, s);
        if (e != hipSuccess) return e;
    } else if (c.n_tiles > 0 && c.n_seg > 0) {
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

hipError_t launch_jacobi_diag(const CacheView& c, const float* gvgram, double* geo, float* M, hipStream_t s) {
    dim3 b(kBlock);
#define LM_D(D)                                                                                          \
    if (c.n_gv > 0) hipLaunchKernelGGL(k_diag_geo_gv<D>, dim3(grid_for(c.n_gv)), b, 0, s, c, gvgram, geo); \
    hipLaunchKernelGGL(k_diag_gauss<D>, dim3(grid_for(c.N)), b, 0, s, c, gvgram, (const double*)geo, M)
    LM_DEG_SWITCH(c.deg, LM_D)
#undef LM_D
    return hipGetLastError();
}

}  // namespace lm
