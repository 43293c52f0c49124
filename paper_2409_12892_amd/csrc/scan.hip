// Device-wide exclusive scan, float64 reduction and a stable LSD radix sort
// of (64- or 32-bit key, 32-bit value) pairs, written for wave64 / 256-thread
// workgroups.  Used by tile binning (depth sort per view, then tile sort),
// the cache build (pair and segment offsets) and the PCG dot products.
#include "lm_internal.h"

namespace lm {
namespace {

constexpr int kScanItems = 16;                       // items per thread
constexpr int kScanTile = kBlock * kScanItems;       // 4096 items per workgroup
// Items per thread of a radix pass: a block ranks kBlock * items keys in LDS
// (more items make longer digit runs but fewer resident blocks; 32 items per
// thread measured slower for both key widths).
template <typename KeyT> constexpr int radix_items() { return 16; }
template <typename KeyT> constexpr int radix_tile() { return kBlock * radix_items<KeyT>(); }
constexpr int kRadixTileMin = kBlock * 16;   // the smallest tile: sizes the scratch

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << __lane_id()) - 1ull;
}

// Inclusive wave scan (wave64) of a 64-bit value.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint64_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive scan across the 256 threads of a block; returns the exclusive
// prefix of `v`, and the block total in *total (same for all threads).
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[kBlock / kWave];
    const int lane = __lane_id();
    const int wid = threadIdx.x / kWave;
    uint64_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        uint64_t s = wsum[w];
        if (w < wid) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__global__ void k_scan_tile_sums(const uint32_t* __restrict__ in, int64_t n, uint64_t* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + (int64_t)i * kBlock + threadIdx.x;
        if (idx < n) acc += in[idx];
    }
    uint64_t tot;
    block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single-workgroup exclusive scan of the tile sums (any length).
__global__ void k_scan_sums(uint64_t* __restrict__ sums, int64_t nb) {
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    uint64_t acc = 0;
    for (int64_t i = 0; i < per; ++i) {
        int64_t idx = b0 + i;
        if (idx < nb) acc += sums[idx];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan(acc, &tot);
    for (int64_t i = 0; i < per; ++i) {
        int64_t idx = b0 + i;
        if (idx < nb) {
            uint64_t s = sums[idx];
            sums[idx] = run;
            run += s;
        }
    }
    if (threadIdx.x == 0) sums[nb] = tot;
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint64_t* __restrict__ sums,
                             uint64_t* __restrict__ out, int64_t nb) {
    // each thread scans kScanItems consecutive items (blocked arrangement)
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0u;
        acc += v[i];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan(acc, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = sums[nb];
}

__global__ void k_reduce_f64(const double* __restrict__ in, int64_t n, double* __restrict__ out) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += in[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---- radix sort ---------------------------------------------------------------
// One pass sorts by a digit of BITS bits (8 or 9; the pass widths of a key
// are chosen so that the passes are as few as 9-bit digits allow), stable:
// per-block digit histograms, one exclusive scan in digit-major order, then
// a scatter that ranks equal digits within a wave by ballots and across the
// block's waves by a prefix of their counts.
template <typename KeyT, int BITS>
__global__ void k_radix_hist(const KeyT* __restrict__ keys, int64_t n, int shift, int64_t nb,
                             uint32_t* __restrict__ hist) {
    constexpr int NDIG = 1 << BITS;
    __shared__ uint32_t h[NDIG];
    for (int d = threadIdx.x; d < NDIG; d += kBlock) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * radix_tile<KeyT>();
#pragma unroll 4
    for (int i = 0; i < radix_items<KeyT>(); ++i) {
        int64_t idx = base + (int64_t)i * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (NDIG - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < NDIG; d += kBlock) hist[(int64_t)d * nb + blockIdx.x] = h[d];   // digit-major
}

// The block's radix_tile items are first ranked by digit in LDS (stable:
// rounds in order, waves in order, lanes in order), then written out in that
// order, so consecutive threads write consecutive addresses of a digit's run.
template <typename KeyT, int BITS>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const KeyT* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals, int64_t n, int shift,
                                                         int64_t nb, const uint64_t* __restrict__ offs,
                                                         KeyT* __restrict__ okeys, uint32_t* __restrict__ ovals) {
    constexpr int NW = kBlock / kWave;
    constexpr int NDIG = 1 << BITS;
    constexpr int DPT = NDIG / kBlock;   // digits owned per thread
    __shared__ uint32_t wcnt[NW][NDIG];
    __shared__ uint32_t lstart[NDIG];    // first local slot of each digit in the block
    __shared__ uint32_t lrun[NDIG];      // items of each digit placed so far
    __shared__ uint64_t s_goff[NDIG];    // global position of the block's first item of each digit
    constexpr int kTile = radix_tile<KeyT>();
    __shared__ KeyT s_key[kTile];
    __shared__ uint32_t s_val[kTile];
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int nloc = (int)(n - base < kTile ? n - base : kTile);
    // the block's count of digit d is the step of the digit-major exclusive
    // scan at (d, block) (its entry past the end holds the total); the local
    // starts are an exclusive scan of those counts over the digits
    {
        uint32_t cnt[DPT];
        uint32_t mine = 0;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int64_t at = (int64_t)(tid * DPT + q) * nb + blockIdx.x;
            const uint64_t o0 = offs[at];
            s_goff[tid * DPT + q] = o0;
            cnt[q] = (uint32_t)(offs[at + 1] - o0);
            mine += cnt[q];
            for (int w = 0; w < NW; ++w) wcnt[w][tid * DPT + q] = 0;
        }
        // exclusive scan of the per-thread sums over the block
        uint32_t inc = mine;
        const int lane = __lane_id();
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        __shared__ uint32_t wsum[NW];
        if (lane == kWave - 1) wsum[wid] = inc;
        __syncthreads();
        uint32_t wbase = 0;
        for (int w = 0; w < wid; ++w) wbase += wsum[w];
        uint32_t run = wbase + inc - mine;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            lstart[tid * DPT + q] = run;
            run += cnt[q];
            lrun[tid * DPT + q] = 0;
        }
        __syncthreads();
    }
    // every round's item is loaded up front (the loads overlap instead of
    // waiting behind each round's barriers)
    KeyT kr[radix_items<KeyT>()];
    uint32_t vr[radix_items<KeyT>()];
#pragma unroll
    for (int r = 0; r < radix_items<KeyT>(); ++r) {
        const int li = r * kBlock + tid;
        kr[r] = li < nloc ? keys[base + li] : (KeyT)0;
        vr[r] = li < nloc ? vals[base + li] : 0u;
    }
#pragma unroll
    for (int r = 0; r < radix_items<KeyT>(); ++r) {
        const int li = r * kBlock + tid;
        const bool live = li < nloc;
        const KeyT k = kr[r];
        const uint32_t v = vr[r];
        const uint32_t d = (uint32_t)((k >> shift) & (NDIG - 1));
        uint64_t peers = __ballot(live);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (live && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t tot[DPT];
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int dg = tid * DPT + q;
            uint32_t c[NW];
            tot[q] = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) c[w] = wcnt[w][dg];
#pragma unroll
            for (int w = 0; w < NW; ++w) { wcnt[w][dg] = tot[q]; tot[q] += c[w]; }
        }
        __syncthreads();
        if (live) {
            const uint32_t slot = lstart[d] + lrun[d] + wcnt[wid][d] + rank;
            s_key[slot] = k;
            s_val[slot] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int dg = tid * DPT + q;
            lrun[dg] += tot[q];
#pragma unroll
            for (int w = 0; w < NW; ++w) wcnt[w][dg] = 0;
        }
        __syncthreads();
    }
    // write the block's items in local digit order
    for (int i = tid; i < nloc; i += kBlock) {
        const KeyT k = s_key[i];
        const uint32_t d = (uint32_t)((k >> shift) & (NDIG - 1));
        const uint64_t pos = s_goff[d] + (uint64_t)(i - (int)lstart[d]);
        okeys[pos] = k;
        ovals[pos] = s_val[i];
    }
}

// out[v] = sum of in[tile_base_v .. tile_base_v + TX TY), one workgroup per view.
__global__ void k_view_sum_f64(const CamDev* __restrict__ cams, const double* __restrict__ in,
                               double* __restrict__ out) {
    __shared__ double red[kBlock / kWave];
    const CamDev& cam = cams[blockIdx.x];
    const int64_t n = (int64_t)cam.TX * cam.TY;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += in[cam.tile_base + i];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (__lane_id() == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += red[w];
        out[blockIdx.x] = tot;
    }
}

}  // namespace

hipError_t view_sum_f64(const CamDev* cams, int V, const double* in, double* out, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_view_sum_f64, dim3((unsigned)V), dim3(kBlock), 0, s, cams, in, out);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(uint64_t);
}

hipError_t exclusive_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, void* tmp,
                                     size_t tmp_bytes, hipStream_t s) {
    if (n <= 0) return hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if ((size_t)(nb + 1) * sizeof(uint64_t) > tmp_bytes) return hipErrorInvalidValue;
    uint64_t* sums = (uint64_t*)tmp;
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums, out, nb);
    return hipGetLastError();
}

hipError_t reduce_f64(const double* in, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(kBlock), 0, s, in, n, out);
    return hipGetLastError();
}

constexpr int kMaxDigitBits = 9;
constexpr int kMaxDigits = 1 << kMaxDigitBits;

size_t radix_tmp_bytes(int64_t n) {
    int64_t nb = (n + kRadixTileMin - 1) / kRadixTileMin;
    size_t hist = (size_t)kMaxDigits * nb * sizeof(uint32_t);
    size_t offs = (size_t)(kMaxDigits * nb + 1) * sizeof(uint64_t);
    size_t scan = scan_tmp_bytes(kMaxDigits * nb);
    return hist + offs + scan + 256;
}

template <typename KeyT>
hipError_t radix_sort_impl(KeyT* keys, uint32_t* vals, KeyT* keys_alt, uint32_t* vals_alt, int64_t n,
                           int begin_bit, int end_bit, void* tmp, size_t tmp_bytes, bool* result_in_alt,
                           hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    int64_t nb = (n + radix_tile<KeyT>() - 1) / radix_tile<KeyT>();
    if (radix_tmp_bytes(n) > tmp_bytes) return hipErrorInvalidValue;
    char* t = (char*)tmp;
    uint32_t* hist = (uint32_t*)t;
    t += (size_t)kMaxDigits * nb * sizeof(uint32_t);
    t = (char*)(((uintptr_t)t + 7) & ~(uintptr_t)7);
    uint64_t* offs = (uint64_t*)t;
    t += (size_t)(kMaxDigits * nb + 1) * sizeof(uint64_t);
    void* stmp = t;
    size_t stmp_bytes = scan_tmp_bytes(kMaxDigits * nb);
    KeyT* ki = keys; uint32_t* vi = vals;
    KeyT* ko = keys_alt; uint32_t* vo = vals_alt;
    bool alt = false;
    // as few passes as 9-bit digits allow, the bits spread evenly over them.
    // A pass narrower than its kernel's digit also sorts by a few bits of the
    // next digit (harmless: every pass is a stable sort, and the next one
    // orders those bits again) or by bits above end_bit (zero in every key).
    const int bits = end_bit - begin_bit;
    const int passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
    int shift = begin_bit;
    for (int pass = 0; pass < passes; ++pass) {
        const int w = (bits - (shift - begin_bit)) / (passes - pass);   // the wider digits last
        hipError_t e;
        if (w > 8) {
            hipLaunchKernelGGL((k_radix_hist<KeyT, 9>), dim3((unsigned)nb), dim3(kBlock), 0, s, ki, n, shift, nb, hist);
            e = exclusive_scan_u32_to_u64(hist, offs, 512 * nb, stmp, stmp_bytes, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_radix_scatter<KeyT, 9>), dim3((unsigned)nb), dim3(kBlock), 0, s, ki, vi, n, shift,
                               nb, offs, ko, vo);
        } else {
            hipLaunchKernelGGL((k_radix_hist<KeyT, 8>), dim3((unsigned)nb), dim3(kBlock), 0, s, ki, n, shift, nb, hist);
            e = exclusive_scan_u32_to_u64(hist, offs, 256 * nb, stmp, stmp_bytes, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_radix_scatter<KeyT, 8>), dim3((unsigned)nb), dim3(kBlock), 0, s, ki, vi, n, shift,
                               nb, offs, ko, vo);
        }
        shift += w;
        std::swap(ki, ko);
        std::swap(vi, vo);
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipGetLastError();
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                            int begin_bit, int end_bit, void* tmp, size_t tmp_bytes, bool* result_in_alt,
                            hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, begin_bit, end_bit, tmp, tmp_bytes,
                                      result_in_alt, s);
}

hipError_t radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                                int begin_bit, int end_bit, void* tmp, size_t tmp_bytes, bool* result_in_alt,
                                hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, begin_bit, end_bit, tmp, tmp_bytes,
                                      result_in_alt, s);
}

}  // namespace lm
