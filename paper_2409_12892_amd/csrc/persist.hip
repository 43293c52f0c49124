// Persistent-kernel PCG for a batch of image subsets (Algorithm 1 per
// subset; section 3.3, "Image Subsampling Scheme").  One cooperative launch
// runs every iteration of every subset of the batch: each workgroup (one
// per resident slot of the chip) loops over the phases of an iteration, and
// a grid-wide barrier separates the phases:
//   1 tangent per (Gaussian, view)
//   2 tile pass, tiles handed out by an atomic counter (J^T J p per tile)
//   3 per-(Gaussian, view) moment sums, 4 their join across waves
//   5 chain per (Gaussian, view), 6 chain per Gaussian with p.g partials
//   7 alpha = r.z / p.g; x += alpha p, r -= alpha g, z = M^-1 r with r.z and
//     r.r partials
//   8 beta = r.z_new / r.z, the stopping test, p = z + beta p
// The float64 scalars are summed from the workgroups' partials by every
// workgroup in the same fixed order, so all workgroups take identical
// decisions (breakdown, stopping) without another barrier; workgroup 0
// records them for the host.  A subset whose loop has ended skips its work
// in every later phase.  The barrier spins on a counter with a time limit:
// one that does not complete within 10 s sets an error flag, and every later
// barrier then passes at once, so the kernel always ends (the host reports
// the error).
#include "products.h"
#include "thin.h"

namespace lm {
namespace {

constexpr uint64_t kBarrierTicks = 1000000000ull;   // 10 s of the 100 MHz real-time counter
constexpr int kTileThin = 3;                        // tile-pass variant of a thinned cache

// Grid-wide barrier: every thread makes its writes visible to the whole
// device, workgroup leaders count in and wait for the count of this barrier,
// then every thread takes the other workgroups' writes.
__device__ __forceinline__ void grid_barrier(uint32_t* bar, uint32_t& target, int32_t* err) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        target += gridDim.x;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(2);
                if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTicks) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
    }
    __syncthreads();
    __threadfence();
}

// Sum over the workgroup of NV doubles per thread in a fixed order; every
// thread receives the sums.
template <int NT, int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV]) {
    __shared__ double s_red[NT / kWave][NV];
    __shared__ double s_out[NV];
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
        if (lane == 0) s_red[wid][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < NT / kWave; ++w) t += s_red[w][threadIdx.x];
        s_out[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = s_out[k];
    __syncthreads();
}

template <int NT, int DEG, int TILE>
__global__ void __launch_bounds__(NT) k_pcg_persistent(const PersistArgs* __restrict__ A_) {
    const PersistArgs& A = *A_;
    const ApplyBatch& Bt = A.B;
    const int nb = Bt.n;
    const int tid = threadIdx.x, wg = blockIdx.x, G = gridDim.x;
    const int64_t gid = (int64_t)wg * NT + tid, gstride = (int64_t)G * NT;
    // per-subset state of Algorithm 1 (identical in every workgroup)
    __shared__ double s_rz[kMaxBatch], s_bb[kMaxBatch], s_rr[kMaxBatch], s_pg[kMaxBatch], s_alpha[kMaxBatch],
        s_beta[kMaxBatch];
    __shared__ int s_stop[kMaxBatch], s_iters[kMaxBatch], s_status[kMaxBatch];
    __shared__ int64_t s_tile;
    if (tid < nb) {
        const PcgState* st = A.v[tid].st;
        s_rz[tid] = st->rz;
        s_bb[tid] = st->bb;
        s_rr[tid] = st->rr;
        s_pg[tid] = st->pg;
        s_alpha[tid] = st->alpha;
        s_beta[tid] = st->beta;
        s_stop[tid] = st->stop;
        s_iters[tid] = st->iters;
        s_status[tid] = st->status;
    }
    __syncthreads();
    uint32_t target = 0;
    const int64_t total_tiles = Bt.tile_off[nb];
    double* part = A.part;   // [kMaxBatch][3][G]

    for (int it = 0; it < A.n_iters; ++it) {
        // 1 tangent
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            const ApplyArgs& a = Bt.a[b];
            for (int64_t gv = gid; gv < a.c.n_gv; gv += gstride) tangent_body<DEG>(a, gv);
        }
        grid_barrier(A.bar, target, A.err);
        // 2 tile pass
        for (;;) {
            if (tid == 0) s_tile = (int64_t)atomicAdd(&A.tile_ctr[it], 1u);
            __syncthreads();
            const int64_t t = s_tile;
            __syncthreads();
            if (t >= total_tiles) break;
            int bi = 0;
            while (bi + 1 < nb && t >= Bt.tile_off[bi + 1]) ++bi;
            if (s_stop[bi]) continue;
            if constexpr (TILE == kTileThin) thin_tile_body<MODE_JTJ>(Bt, t);
            else apply_tile_body<MODE_JTJ, TILE>(Bt, t);
            __syncthreads();
        }
        grid_barrier(A.bar, target, A.err);
        // 3, 4 moment sums per (Gaussian, view)
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            const ApplyArgs& a = Bt.a[b];
            const int64_t nw = (a.c.n_seg + kWave - 1) / kWave;
            for (int64_t i = gid; i < nw * kWave; i += gstride)
                gv_reduce_body<9>(a.c, a.gmom, a.gvsum, a.edge, a.edge_key, i);
        }
        grid_barrier(A.bar, target, A.err);
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            const ApplyArgs& a = Bt.a[b];
            const int64_t nw = (a.c.n_seg + kWave - 1) / kWave;
            for (int64_t w = gid; w < nw; w += gstride) gv_reduce_join_body<9>(a.c, a.edge, a.edge_key, a.gvsum, w);
        }
        grid_barrier(A.bar, target, A.err);
        // 5, 6 chain, p.g partials
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            const ApplyArgs& a = Bt.a[b];
            for (int64_t gv = gid; gv < a.c.n_gv; gv += gstride) chain_gv_body<DEG>(a, gv);
        }
        grid_barrier(A.bar, target, A.err);
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            const ApplyArgs& a = Bt.a[b];
            double pg[1] = {0.0};
            for (int64_t g = gid; g < a.c.N; g += gstride) pg[0] += chain_body<DEG>(Bt, a, g);
            wg_sum<NT, 1>(pg);
            if (tid == 0) part[(int64_t)(3 * b) * G + wg] = pg[0];
        }
        grid_barrier(A.bar, target, A.err);
        // 7 alpha and the x, r, z update
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            double pg[1] = {0.0};
            for (int j = tid; j < G; j += NT) pg[0] += part[(int64_t)(3 * b) * G + j];
            wg_sum<NT, 1>(pg);
            if (tid == 0) {
                s_pg[b] = pg[0];
                if (!(pg[0] > 0.0) || !isfinite(pg[0])) {
                    s_stop[b] = 1;
                    s_status[b] = LM_WARN_BREAKDOWN;
                } else {
                    s_alpha[b] = s_rz[b] / pg[0];
                }
            }
            __syncthreads();
            if (s_stop[b]) continue;
            const PersistSubset& v = A.v[b];
            const ApplyArgs& a = Bt.a[b];
            const float alpha = (float)s_alpha[b];
            double acc[2] = {0.0, 0.0};
            for (int64_t i = gid; i < A.n; i += gstride) {
                v.x[i] = v.x[i] + alpha * a.p[i];
                const float ri = v.r[i] - alpha * a.out[i];
                const float zi = jacobi_inv(v.M[i], A.floor_, v.scale, i) * ri;
                v.r[i] = ri;
                v.z[i] = zi;
                acc[0] += (double)ri * zi;
                acc[1] += (double)ri * ri;
            }
            wg_sum<NT, 2>(acc);
            if (tid == 0) {
                part[(int64_t)(3 * b + 1) * G + wg] = acc[0];
                part[(int64_t)(3 * b + 2) * G + wg] = acc[1];
            }
        }
        grid_barrier(A.bar, target, A.err);
        // 8 beta, the stopping test, p = z + beta p
        for (int b = 0; b < nb; ++b) {
            if (s_stop[b]) continue;
            double s2[2] = {0.0, 0.0};
            for (int j = tid; j < G; j += NT) {
                s2[0] += part[(int64_t)(3 * b + 1) * G + j];
                s2[1] += part[(int64_t)(3 * b + 2) * G + j];
            }
            wg_sum<NT, 2>(s2);
            if (tid == 0) {
                const double rz_new = s2[0], rr = s2[1];
                s_beta[b] = s_rz[b] != 0.0 ? rz_new / s_rz[b] : 0.0;
                s_rz[b] = rz_new;
                s_rr[b] = rr;
                const int k = s_iters[b] + 1;
                s_iters[b] = k;
                if (wg == 0 && k < LM_PCG_MAX_HISTORY) A.v[b].st->hist[k] = s_bb[b] > 0.0 ? rr / s_bb[b] : 0.0;
                if (A.tol_mode == LM_TOL_PAPER_SQUARED && rr < A.tol * s_bb[b]) s_stop[b] = 1;
                if (A.tol_mode == LM_TOL_RELATIVE && sqrt(rr) < A.tol * sqrt(s_bb[b])) s_stop[b] = 1;
            }
            __syncthreads();
            if (s_stop[b]) continue;
            const float beta = (float)s_beta[b];
            const PersistSubset& v = A.v[b];
            for (int64_t i = gid; i < A.n; i += gstride) v.p[i] = v.z[i] + beta * v.p[i];
        }
        grid_barrier(A.bar, target, A.err);
    }
    if (wg == 0 && tid < nb) {
        PcgState* st = A.v[tid].st;
        st->rz = s_rz[tid];
        st->rr = s_rr[tid];
        st->pg = s_pg[tid];
        st->alpha = s_alpha[tid];
        st->beta = s_beta[tid];
        st->stop = s_stop[tid];
        st->iters = s_iters[tid];
        st->status = s_status[tid];
    }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

template <int NT, int DEG, int TILE>
const void* persistent_kernel() {
    return reinterpret_cast<const void*>(&k_pcg_persistent<NT, DEG, TILE>);
}

// the kernel of a (SH degree, tile variant) pair and its workgroup size
const void* persistent_select(int deg, int tile, int* nt) {
#define LM_PK(D)                                                                          \
    if (deg == D) {                                                                       \
        if (tile == kTileThin) { *nt = kThinThreads; return persistent_kernel<kThinThreads, D, kTileThin>(); } \
        *nt = kTileThreads;                                                               \
        if (tile == LM_CACHE_F32) return persistent_kernel<kTileThreads, D, LM_CACHE_F32>(); \
        if (tile == LM_CACHE_BF16) return persistent_kernel<kTileThreads, D, LM_CACHE_BF16>(); \
        return persistent_kernel<kTileThreads, D, LM_CACHE_F16>();                         \
    }
    LM_PK(0)
    LM_PK(1)
    LM_PK(2)
    LM_PK(3)
#undef LM_PK
    return nullptr;
}

}  // namespace

int persistent_tile_kind(int dtype, bool thin) { return thin ? kTileThin : dtype; }

hipError_t persistent_grid(int deg, int tile, int* grid, int* nt) {
    const void* k = persistent_select(deg, tile, nt);
    if (!k) return hipErrorInvalidValue;
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, *nt, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    *grid = std::min(per_cu * ncu, kPersistMaxGrid);
    return hipSuccess;
}

hipError_t launch_pcg_persistent(const PersistArgs* dev_args, uint32_t* counters, int n_counters, int deg, int tile,
                                 int grid, hipStream_t s) {
    int nt = 0;
    const void* k = persistent_select(deg, tile, &nt);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBlock), 0, s, counters, n_counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&dev_args};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(nt), args, 0, s);
}

}  // namespace lm
