// Projection of every (Gaussian, view) in float64 and tile binning.
//
// Binning is an integer function of float32 records: mean and depth are the
// float64 projection rounded to float32, the tile rectangle is
// floor((m -/+ r) / tile) evaluated in float32 (IEEE division) with inclusive
// bounds, and each tile's list is ordered by (float32 depth bits, Gaussian
// id).  The order is reached in two stable sorts: the binned records of all
// views by (view, depth bits) (records start in (view, id) order, and depth
// > 0.2 has a zero sign bit), then the keys - emitted record by record in
// that order - by global tile index alone.
#include "proj_math.h"

namespace lm {
namespace {

__device__ __forceinline__ void tile_rect(float mx, float my, int32_t radius, int TW, int TH, int TX, int TY,
                                          int& x0, int& y0, int& x1, int& y1) {
    const float r = (float)radius;
    const float fx0 = floorf(__fdiv_rn(mx - r, (float)TW));
    const float fx1 = floorf(__fdiv_rn(mx + r, (float)TW));
    const float fy0 = floorf(__fdiv_rn(my - r, (float)TH));
    const float fy1 = floorf(__fdiv_rn(my + r, (float)TH));
    x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)TX);
    x1 = (int)fmaxf(fminf(fx1, (float)(TX - 1)), -1.0f);
    y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)TY);
    y1 = (int)fmaxf(fminf(fy1, (float)(TY - 1)), -1.0f);
}

// Largest exponent -0.5 (A dx^2 + 2 B dx dy + C dy^2) of a splat over the
// box [xa, xb] x [ya, yb] of offsets from its mean (the pixel centres of a
// tile): 0 when the mean lies inside, else the best point of the four
// edges (the exponent is concave; iA = 1 / A, iC = 1 / C).  Evaluated
// without contracted multiply-adds, in a fixed order, so that it is a
// reproducible function of its float64 inputs.
__device__ __forceinline__ double tile_max_power(double A, double B, double C, double iA, double iC, double xa,
                                                 double xb, double ya, double yb) {
#pragma clang fp contract(off)
    if (xa <= 0.0 && 0.0 <= xb && ya <= 0.0 && 0.0 <= yb) return 0.0;
    double best = -INFINITY;
    const double xe[2] = {xa, xb}, ye[2] = {ya, yb};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double xx = xe[k];
        const double yy = fmin(fmax(-(B * xx) * iC, ya), yb);
        best = fmax(best, -0.5 * (A * xx * xx + 2.0 * B * xx * yy + C * yy * yy));
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double yy = ye[k];
        const double xx = fmin(fmax(-(B * yy) * iA, xa), xb);
        best = fmax(best, -0.5 * (A * xx * xx + 2.0 * B * xx * yy + C * yy * yy));
    }
    return best;
}

template <int deg>
__device__ __forceinline__ void project_one(const CamDev* __restrict__ cams, const float* __restrict__ x, int64_t N,
                                            int V, int TW, int TH, int64_t r, float* __restrict__ recf,
                                            int32_t* __restrict__ rad, uint32_t* __restrict__ keycnt,
                                            double* __restrict__ rec) {
    const int64_t R = N * (int64_t)V;
    const int v = (int)(r / N);
    const int64_t g = r - (int64_t)v * N;
    const CamDev& cam = cams[v];
    ProjFwd f;
    proj_forward<deg>(cam, x, N, g, f);
    uint32_t cnt = 0;
    const float mx32 = (float)f.mx, my32 = (float)f.my, z32 = (float)f.z;
    if (f.vis) {
        int x0, y0, x1, y1;
        tile_rect(mx32, my32, f.radius, TW, TH, cam.TX, cam.TY, x0, y0, x1, y1);
        if (x0 <= x1 && y0 <= y1) cnt = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    }
    keycnt[r] = cnt;
    rad[r] = f.vis ? f.radius : 0;
    recf[r] = mx32;
    recf[R + r] = my32;
    recf[2 * R + r] = z32;
    const double o = f.o;
    const double vals[10] = {f.mx, f.my, f.A, f.B, f.C, o, -log(255.0 * o), f.col[0], f.col[1], f.col[2]};
#pragma unroll
    for (int i = 0; i < 10; ++i) rec[i] = vals[i];
#pragma unroll
    for (int i = 10; i < kRecStride; ++i) rec[i] = 0.0;
}

// rec64 layout [V*N][kRecStride]: mx, my, A, B, C, o, log threshold, r, g, b (float64)
template <int deg>
__global__ void k_project(const CamDev* __restrict__ cams, const float* __restrict__ x, int64_t N, int V,
                          int TW, int TH, double* __restrict__ rec64, float* __restrict__ recf,
                          int32_t* __restrict__ rad, uint32_t* __restrict__ keycnt) {
    const int64_t R = N * (int64_t)V;
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t r = r0 + threadIdx.x;
    // the block's records go through LDS (rows padded by one double against
    // bank conflicts) and leave as one contiguous run
    constexpr int kRow = kRecStride + 1;
    __shared__ double s_rec[kBlock * kRow];
    if (r < R) project_one<deg>(cams, x, N, V, TW, TH, r, recf, rad, keycnt, &s_rec[threadIdx.x * kRow]);
    __syncthreads();
    const int nrec = (int)(R - r0 < kBlock ? R - r0 : kBlock);
    double* dst = rec64 + r0 * kRecStride;
    for (int i = threadIdx.x; i < nrec * kRecStride; i += kBlock) dst[i] = s_rec[(i / kRecStride) * kRow + i % kRecStride];
}



// Depth-sort key of every record: (view << 31) | float32 depth bits for a
// binned record, (view << 31) | 0x7FFFFFFF for one that emits no key.
__global__ void k_record_keys(const float* __restrict__ recf, const uint32_t* __restrict__ keycnt, int64_t N,
                              int V, uint64_t* __restrict__ rkeys, uint32_t* __restrict__ rvals) {
    const int64_t R = N * (int64_t)V;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint64_t v = (uint64_t)(r / N);
    const uint32_t zb = keycnt[r] > 0 ? __float_as_uint(recf[2 * R + r]) : 0x7FFFFFFFu;
    rkeys[r] = (v << 31) | zb;
    rvals[r] = (uint32_t)r;
}

__global__ void k_gather_counts(const uint32_t* __restrict__ order, const uint32_t* __restrict__ keycnt, int64_t R,
                                uint32_t* __restrict__ cnt_sorted) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) cnt_sorted[i] = keycnt[order[i]];
}

// Keys (global tile index) and values (Gaussian id) of the records in depth
// order; record order[i] writes its tiles (row by row) at off_sorted[i].
// A tile of the rectangle in which the splat's exponent stays below its
// alpha threshold (alpha < 1/255) by a margin at every pixel centre is left
// out.  Two launches: COUNT evaluates the test, stores each wave's ballot of
// kept keys in kept_mask and counts each block's kept keys; after a scan of
// the counts the emitting launch reads the ballots back and writes the kept
// keys contiguously, in the same order (each round of 256 keys ranked with
// the ballots).  Block b's ballots start at word b0/64 + 5b (b0 its first
// key), one word per wave and round: the regions of consecutive blocks do
// not overlap, and all fit in bin_mask_words(K, R) words.
// A block takes 256 consecutive records and writes their keys together:
// each thread takes every 256th key of the block's range and finds its
// record by a fixed-step search over the block's offsets, so the stores of
// a wave are consecutive.
template <bool COUNT>
__global__ void __launch_bounds__(kBlock) k_bin_emit(const CamDev* __restrict__ cams, int64_t N, int64_t R, int TW,
                                                    int TH, const float* __restrict__ recf,
                                                    const int32_t* __restrict__ rad,
                                                    const uint32_t* __restrict__ order,
                                                    const uint64_t* __restrict__ off_sorted,
                                                    const double* __restrict__ rec64,
                                                    uint64_t* __restrict__ kept_mask,
                                                    uint32_t* __restrict__ kept_blk,
                                                    const uint64_t* __restrict__ kept_off, uint64_t n_kept,
                                                    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_off[kBlock];    // first key of each record, relative to the block
    __shared__ int32_t s_x0[kBlock], s_y0[kBlock], s_w[kBlock];
    __shared__ uint32_t s_base[kBlock], s_g[kBlock], s_tx[kBlock];
    __shared__ double s_iA[kBlock], s_iC[kBlock], s_q[6][kBlock];   // q: mx, my, A, B, C, log threshold
    __shared__ uint32_t s_wsum[kBlock / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = i0 + threadIdx.x;
    const int64_t ie = i0 + kBlock < R ? i0 + kBlock : R;
    const uint64_t b0 = off_sorted[i0], b1 = off_sorted[ie];
    // records that emit no key sort last in their view: most blocks have none
    if (b0 == b1) {
        if (COUNT && threadIdx.x == 0) kept_blk[blockIdx.x] = 0;
        return;
    }
    if (i < R) {
        const int64_t r = order[i];
        const int v = (int)(r / N);
        const CamDev& cam = cams[v];
        int x0, y0, x1, y1;
        tile_rect(recf[r], recf[R + r], rad[r], TW, TH, cam.TX, cam.TY, x0, y0, x1, y1);
        s_off[threadIdx.x] = (uint32_t)(off_sorted[i] - b0);
        s_x0[threadIdx.x] = x0;
        s_y0[threadIdx.x] = y0;
        s_w[threadIdx.x] = x1 - x0 + 1;
        s_base[threadIdx.x] = (uint32_t)cam.tile_base;
        s_tx[threadIdx.x] = (uint32_t)cam.TX;
        s_g[threadIdx.x] = (uint32_t)(r - (int64_t)v * N);
        if (COUNT) {
            const double* rc = rec64 + r * kRecStride;
#pragma unroll
            for (int q = 0; q < 5; ++q) s_q[q][threadIdx.x] = rc[q];
            s_q[5][threadIdx.x] = rc[6];
            s_iA[threadIdx.x] = 1.0 / rc[2];
            s_iC[threadIdx.x] = 1.0 / rc[4];
        }
    } else {
        s_off[threadIdx.x] = (uint32_t)(b1 - b0);   // past the block's last key: never selected
    }
    __syncthreads();
    const uint32_t nk = (uint32_t)(b1 - b0);
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
    const uint64_t base = COUNT ? 0 : kept_off[blockIdx.x];
    uint64_t* const mask = kept_mask + (b0 / kWave + 5 * (uint64_t)blockIdx.x) + wid;
    uint32_t running = 0;
    // key k's tile, Gaussian and (COUNT) tile test
    auto key_at = [&](uint32_t k, uint32_t& key, uint32_t& val, bool& keep) {
        keep = false;
        key = val = 0;
        if (k >= nk) return;
        // the last record whose first key is at or before k holds key k
        // (s_off ascends from s_off[0] = 0; fixed-step search)
        int lo = 0;
#pragma unroll
        for (int step = kBlock / 2; step > 0; step >>= 1) lo = s_off[lo + step] <= k ? lo + step : lo;
        const uint32_t j = k - s_off[lo];
        const int w = s_w[lo];
        const int ty = s_y0[lo] + (int)(j / (uint32_t)w), tx = s_x0[lo] + (int)(j % (uint32_t)w);
        if (COUNT) {
            const double xa = ((double)(tx * TW) + 0.5) - s_q[0][lo];
            const double ya = ((double)(ty * TH) + 0.5) - s_q[1][lo];
            const double pmax = tile_max_power(s_q[2][lo], s_q[3][lo], s_q[4][lo], s_iA[lo], s_iC[lo], xa,
                                               xa + (double)(TW - 1), ya, ya + (double)(TH - 1));
            keep = !(pmax < s_q[5][lo] - kCullMargin);
        }
        key = s_base[lo] + (uint32_t)ty * s_tx[lo] + (uint32_t)tx;
        val = s_g[lo];
    };
    // every wave runs every round of the block; a thread takes one key of
    // each of kRounds rounds per iteration (independent searches in flight)
    constexpr int kRounds = 2;
    for (uint32_t k0 = 0; k0 < nk; k0 += kRounds * kBlock) {
        uint32_t key[kRounds], val[kRounds];
        bool keep[kRounds];
#pragma unroll
        for (int h = 0; h < kRounds; ++h) key_at(k0 + h * kBlock + threadIdx.x, key[h], val[h], keep[h]);
#pragma unroll
        for (int h = 0; h < kRounds; ++h) {
            const uint32_t kr = k0 + h * kBlock;   // the round's first key
            if (kr >= nk) break;
            const uint32_t round = kr / kBlock;
            if (COUNT) {
                const uint64_t m = (uint64_t)__ballot(keep[h]);
                if (lane == 0) mask[4 * round] = m;
                running += (uint32_t)__popcll(m);
            } else {
                // the round's four ballots: this wave's keys and the kept
                // keys of the waves before it
                const uint64_t* rw = mask - wid + 4 * round;
                uint32_t before = 0, total = 0;
                uint64_t m = 0;
#pragma unroll
                for (int w = 0; w < kBlock / kWave; ++w) {
                    const uint64_t mw = rw[w];
                    const uint32_t c = (uint32_t)__popcll(mw);
                    before += w < wid ? c : 0u;
                    total += c;
                    m = w == wid ? mw : m;
                }
                if ((m >> lane) & 1ull) {
                    const uint64_t pos = base + running + before + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                    if (pos < n_kept) {
                        keys[pos] = key[h];
                        vals[pos] = val[h];
                    }
                }
                running += total;
            }
        }
    }
    if (COUNT) {
        // the block's kept keys: the sum of its waves' counts
        if (lane == 0) s_wsum[wid] = running;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < kBlock / kWave; ++w) t += s_wsum[w];
            kept_blk[blockIdx.x] = t;
        }
    }
}

// tile_start[t] = first key index of tile t (lists are [tile_start[t], tile_start[t+1])).
// Grid-stride over the keys: a launch's work-item count is a 32-bit number,
// and the key count of a large subset exceeds it.
__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, int64_t K, int64_t n_tiles,
                              int64_t* __restrict__ tile_start) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = (int64_t)keys[i];
        const int64_t tp = i == 0 ? -1 : (int64_t)keys[i - 1];
        for (int64_t u = tp + 1; u <= t; ++u) tile_start[u] = i;
        if (i == K - 1)
            for (int64_t u = t + 1; u <= n_tiles; ++u) tile_start[u] = K;
    }
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_project(const CamDev* cams, const float* x, int64_t N, int V, int deg, int TW, int TH,
                          double* rec64, float* recf, int32_t* rad, uint32_t* keycnt, hipStream_t s) {
    const int64_t R = N * (int64_t)V;
    switch (deg) {
        case 0: hipLaunchKernelGGL(k_project<0>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, x, N, V, TW, TH, rec64,
                                   recf, rad, keycnt); break;
        case 1: hipLaunchKernelGGL(k_project<1>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, x, N, V, TW, TH, rec64,
                                   recf, rad, keycnt); break;
        case 2: hipLaunchKernelGGL(k_project<2>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, x, N, V, TW, TH, rec64,
                                   recf, rad, keycnt); break;
        default: hipLaunchKernelGGL(k_project<3>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, x, N, V, TW, TH, rec64,
                                    recf, rad, keycnt); break;
    }
    return hipGetLastError();
}

hipError_t launch_record_keys(const float* recf, const uint32_t* keycnt, int64_t N, int V, uint64_t* rkeys,
                              uint32_t* rvals, hipStream_t s) {
    const int64_t R = N * (int64_t)V;
    hipLaunchKernelGGL(k_record_keys, dim3(grid_for(R)), dim3(kBlock), 0, s, recf, keycnt, N, V, rkeys, rvals);
    return hipGetLastError();
}

hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* keycnt, int64_t R, uint32_t* cnt_sorted,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_gather_counts, dim3(grid_for(R)), dim3(kBlock), 0, s, order, keycnt, R, cnt_sorted);
    return hipGetLastError();
}

int64_t bin_emit_blocks(int64_t R) { return grid_for(R); }

// block b's last ballot word is below (b0 + nk)/64 + 5b + 4 <= K/64 + 5 nblocks
int64_t bin_mask_words(int64_t K, int64_t R) { return K / kWave + 5 * bin_emit_blocks(R) + 8; }

hipError_t launch_bin_count(const CamDev* cams, int64_t N, int64_t R, int TW, int TH, const float* recf,
                            const int32_t* rad, const uint32_t* order, const uint64_t* off_sorted,
                            const double* rec64, uint64_t* kept_mask, uint32_t* kept_blk, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_emit<true>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, N, R, TW, TH, recf, rad, order,
                       off_sorted, rec64, kept_mask, kept_blk, nullptr, (uint64_t)0, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_bin_emit(const CamDev* cams, int64_t N, int64_t R, int TW, int TH, const float* recf,
                           const int32_t* rad, const uint32_t* order, const uint64_t* off_sorted,
                           const double* rec64, uint64_t* kept_mask, const uint64_t* kept_off, int64_t n_kept,
                           uint32_t* keys, uint32_t* vals, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_emit<false>, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, N, R, TW, TH, recf, rad, order,
                       off_sorted, rec64, kept_mask, nullptr, kept_off, (uint64_t)n_kept, keys, vals);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* keys, int64_t K, int64_t n_tiles, int64_t* tile_start,
                              hipStream_t s) {
    if (K == 0) {
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_tiles + 1)), dim3(kBlock), 0, s, tile_start, n_tiles + 1,
                           (int64_t)0);
    } else {
        const unsigned grid = std::min<unsigned>(grid_for(K), 1u << 20);
        hipLaunchKernelGGL(k_tile_ranges, dim3(grid), dim3(kBlock), 0, s, keys, K, n_tiles, tile_start);
    }
    return hipGetLastError();
}

}  // namespace lm
