// Vector half of Algorithm 1 (PCG) with float64 dot products and scalars
// kept on the device, and the subset combination (eq. combine-pcg).
//
// Every kernel of an iteration reads the device `stop` flag first and
// returns when it is set, so the host enqueues n_iters iterations without
// synchronising and the loop still ends where Algorithm 1 breaks.
#include "lm_internal.h"

namespace lm {



namespace {

constexpr int kVecBlocks = 2048;   // fixed grid: partial sums in a fixed order

// M^-1 of Algorithm 1 with the optional minimum diagonal (0 where M = 0).
__device__ __forceinline__ float jacobi_inv(float M, float floor_, const float* scale, int64_t i) {
    if (!(M > 0.0f)) return 0.0f;
    const float s = scale ? scale[i] : 1.0f;
    return s / fmaxf(M, floor_);
}

template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* part, int64_t stride) {
    __shared__ double sh[NV][kBlock / kWave];
    const int lane = __lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
        if (lane == 0) sh[k][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += sh[k][w];
            part[k * stride + blockIdx.x] = s;
        }
    }
}

__device__ double block_sum(const double* part, int64_t n) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// x0 = M^-1 b
__global__ void k_init_x(int64_t n, const float* __restrict__ b, const float* __restrict__ M, float floor_,
                         const float* __restrict__ scale, float* __restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = jacobi_inv(M[i], floor_, scale, i) * b[i];
}

// r0 = b - g, z0 = M^-1 r0, p0 = z0; partials of r.z, r.r, b.b
__global__ void k_init_r(int64_t n, const float* __restrict__ b, const float* __restrict__ g,
                         const float* __restrict__ M, float floor_, const float* __restrict__ scale, float* __restrict__ r,
                         float* __restrict__ z, float* __restrict__ p, double* __restrict__ part) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float ri = b[i] - g[i];
        const float zi = jacobi_inv(M[i], floor_, scale, i) * ri;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        acc[0] += (double)ri * zi;
        acc[1] += (double)ri * ri;
        acc[2] += (double)b[i] * b[i];
    }
    block_partials<3>(acc, part, gridDim.x);
}

__global__ void k_init_scalars(const double* __restrict__ part, int64_t nb, PcgState* st) {
    const double rz = block_sum(part, nb);
    const double rr = block_sum(part + nb, nb);
    const double bb = block_sum(part + 2 * nb, nb);
    if (threadIdx.x == 0) {
        st->rz = rz;
        st->rr = rr;
        st->bb = bb;
        st->iters = 0;
        st->status = 0;
        st->stop = 0;
        st->hist[0] = bb > 0.0 ? rr / bb : 0.0;
    }
}

// alpha = r.z / p.g, with a breakdown stop when p.g is not positive and finite
__global__ void k_alpha(const double* __restrict__ pg_part, int64_t nb, PcgState* st) {
    if (st->stop) return;
    const double pg = block_sum(pg_part, nb);
    if (threadIdx.x == 0) {
        st->pg = pg;
        if (!(pg > 0.0) || !isfinite(pg)) {
            st->stop = 1;
            st->status = LM_WARN_BREAKDOWN;
        } else {
            st->alpha = st->rz / pg;
        }
    }
}

// x += alpha p, r -= alpha g, z = M^-1 r; partials of r.z and r.r
__global__ void k_update_xrz(int64_t n, const PcgState* __restrict__ st, const float* __restrict__ p,
                             const float* __restrict__ g, const float* __restrict__ M, float floor_,
                             const float* __restrict__ scale, float* __restrict__ x, float* __restrict__ r,
                             float* __restrict__ z, double* __restrict__ part) {
    if (st->stop) return;
    const float alpha = (float)st->alpha;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = x[i] + alpha * p[i];
        const float ri = r[i] - alpha * g[i];
        const float zi = jacobi_inv(M[i], floor_, scale, i) * ri;
        r[i] = ri;
        z[i] = zi;
        acc[0] += (double)ri * zi;
        acc[1] += (double)ri * ri;
    }
    block_partials<2>(acc, part, gridDim.x);
}

// beta = r_new.z_new / r.z; history; stopping rule of Algorithm 1
__global__ void k_beta(const double* __restrict__ part, int64_t nb, PcgState* st, double tol, int tol_mode) {
    if (st->stop) return;
    const double rz_new = block_sum(part, nb);
    const double rr = block_sum(part + nb, nb);
    if (threadIdx.x == 0) {
        st->beta = st->rz != 0.0 ? rz_new / st->rz : 0.0;
        st->rz = rz_new;
        st->rr = rr;
        const int it = st->iters + 1;
        st->iters = it;
        if (it < LM_PCG_MAX_HISTORY) st->hist[it] = st->bb > 0.0 ? rr / st->bb : 0.0;
        if (tol_mode == LM_TOL_PAPER_SQUARED && rr < tol * st->bb) st->stop = 1;
        if (tol_mode == LM_TOL_RELATIVE && sqrt(rr) < tol * sqrt(st->bb)) st->stop = 1;
    }
}

// p = z + beta p
__global__ void k_update_p(int64_t n, const PcgState* __restrict__ st, const float* __restrict__ z,
                           float* __restrict__ p) {
    if (st->stop) return;
    const float beta = (float)st->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

// ---- block-Jacobi preconditioner ------------------------------------------
// Per Gaussian the damped block A_k = B_k + lambda diag(max(d, floor)) of
// the normal equations restricted to its own parameters (d = diag(B_k); a
// parameter with d = 0 keeps a unit diagonal and no coupling), factored
// A_k = L_k L_k^T and stored packed lower row-major, L[g][i (i + 1) / 2 + j].

// One wave per Gaussian: the dense block of a chunk is staged in LDS as
// float64, damped and factored (right-looking, lane i owns row i); a
// non-positive pivot falls back to the block's damped diagonal.
template <int P>
__global__ void __launch_bounds__(kWave) k_bj_factor(const float* __restrict__ blocks, int64_t g0, int64_t n,
                                                    float lam, float floor_, float* __restrict__ L,
                                                    uint32_t* __restrict__ n_fallback) {
    constexpr int T = P * (P + 1) / 2;
    __shared__ double A[P][P + 1];
    __shared__ double sdd[P];
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const float* Bk = blocks + s * P * P;
    for (int i = lane; i < P * P; i += kWave) A[i / P][i % P] = (double)Bk[i];
    __syncthreads();
    const double d = lane < P ? A[lane < P ? lane : 0][lane < P ? lane : 0] : 0.0;
    const uint64_t obs = __ballot(lane < P && d > 0.0);
    __syncthreads();
    for (int i = lane; i < P * P; i += kWave) {
        const int r = i / P, c = i % P;
        if (!((obs >> r) & 1) || !((obs >> c) & 1)) A[r][c] = 0.0;
    }
    __syncthreads();
    const double dd = lane < P ? (d > 0.0 ? d + (double)lam * fmax(d, (double)floor_) : 1.0) : 1.0;
    if (lane < P) {
        A[lane][lane] = dd;
        sdd[lane] = dd;
    }
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < P; ++k) {
        const double akk = A[k][k];
        if (!(akk > 0.0) || !isfinite(akk)) {
            ok = false;
            break;
        }
        const double lkk = sqrt(akk);
        __syncthreads();
        if (lane == k) A[k][k] = lkk;
        if (lane > k && lane < P) A[lane][k] /= lkk;
        __syncthreads();
        if (lane > k && lane < P) {
            const double lik = A[lane][k];
            for (int j = k + 1; j <= lane; ++j) A[lane][j] -= lik * A[j][k];
        }
        __syncthreads();
    }
    float* Lg = L + (g0 + s) * T;
    for (int t = lane; t < T; t += kWave) {
        int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        while (i * (i + 1) / 2 > t) --i;
        const int j = t - i * (i + 1) / 2;
        // without a factorisation: the damped diagonal alone (Jacobi on
        // this Gaussian)
        Lg[t] = ok ? (float)A[i][j] : (i == j ? (float)sqrt(sdd[i]) : 0.0f);
    }
    if (!ok && lane == 0) atomicAdd(n_fallback, 1u);
}

// z = A^-1 r per Gaussian, one wave per Gaussian over a fixed grid (the PCG
// partial grid): the factor goes to LDS, lane j holds entry j, and the
// forward and backward substitutions broadcast each solved entry.  Writes
// z (and a copy to z2 when given) and the block partials of r . z.
template <int P>
__global__ void __launch_bounds__(kBlock) k_bj_solve(const float* __restrict__ L, int64_t N,
                                                   const float* __restrict__ r, float* __restrict__ z,
                                                   float* __restrict__ z2, double* __restrict__ part,
                                                   const PcgState* __restrict__ st) {
    if (st && st->stop) return;
    constexpr int T = P * (P + 1) / 2;
    constexpr int NW = kBlock / kWave;
    __shared__ float sL[NW][T];
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    double acc[1] = {0.0};
    for (int64_t g = (int64_t)blockIdx.x * NW + w; g < N; g += (int64_t)gridDim.x * NW) {
        const float* Lg = L + g * T;
        for (int t = lane; t < T; t += kWave) sL[w][t] = Lg[t];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float rj = lane < P ? r[(int64_t)lane * N + g] : 0.0f;
        float y = rj;
        for (int k = 0; k < P; ++k) {
            const float yk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), k)) /
                             sL[w][k * (k + 1) / 2 + k];
            if (lane == k) y = yk;
            else if (lane > k && lane < P) y -= sL[w][lane * (lane + 1) / 2 + k] * yk;
        }
        for (int k = P - 1; k >= 0; --k) {
            const float zk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), k)) /
                             sL[w][k * (k + 1) / 2 + k];
            if (lane == k) y = zk;
            else if (lane < k) y -= sL[w][k * (k + 1) / 2 + lane] * zk;
        }
        if (lane < P) {
            z[(int64_t)lane * N + g] = y;
            if (z2) z2[(int64_t)lane * N + g] = y;
            acc[0] += (double)rj * y;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (part) block_partials<1>(acc, part, gridDim.x);
}

template <int P>
hipError_t bj_solve_p(const BlockPrecond& bj, const float* r, float* z, float* z2, double* part, const PcgState* st,
                      unsigned nb, hipStream_t s) {
    hipLaunchKernelGGL(k_bj_solve<P>, dim3(nb), dim3(kBlock), 0, s, bj.L, bj.N, r, z, z2, part, st);
    return hipGetLastError();
}

hipError_t bj_solve(const BlockPrecond& bj, const float* r, float* z, float* z2, double* part, const PcgState* st,
                    unsigned nb, hipStream_t s) {
    switch (bj.P) {
        case 14: return bj_solve_p<14>(bj, r, z, z2, part, st, nb, s);
        case 23: return bj_solve_p<23>(bj, r, z, z2, part, st, nb, s);
        case 38: return bj_solve_p<38>(bj, r, z, z2, part, st, nb, s);
        case 59: return bj_solve_p<59>(bj, r, z, z2, part, st, nb, s);
        default: return hipErrorInvalidValue;
    }
}

struct CombineArgs {
    const float* d[16];
    const float* m[16];
    int nb;
};

__global__ void k_combine(CombineArgs a, int64_t n, float* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double num = 0.0, den = 0.0;
        for (int k = 0; k < a.nb; ++k) {
            const double w = a.m[k][i];
            num += w * (double)a.d[k][i];
            den += w;
        }
        out[i] = den > 0.0 ? (float)(num / den) : 0.0f;
    }
}

unsigned vec_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kVecBlocks) g = kVecBlocks;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int64_t pcg_partial_count(int64_t n) { return vec_grid(n); }

hipError_t launch_bj_factor(const float* blocks, int P, int64_t g0, int64_t n, float lam, float floor_, float* L,
                            uint32_t* n_fallback, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)n), b(kWave);
    switch (P) {
        case 14: hipLaunchKernelGGL(k_bj_factor<14>, g, b, 0, s, blocks, g0, n, lam, floor_, L, n_fallback); break;
        case 23: hipLaunchKernelGGL(k_bj_factor<23>, g, b, 0, s, blocks, g0, n, lam, floor_, L, n_fallback); break;
        case 38: hipLaunchKernelGGL(k_bj_factor<38>, g, b, 0, s, blocks, g0, n, lam, floor_, L, n_fallback); break;
        case 59: hipLaunchKernelGGL(k_bj_factor<59>, g, b, 0, s, blocks, g0, n, lam, floor_, L, n_fallback); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bj_apply(const BlockPrecond& bj, const float* r, float* z, hipStream_t s) {
    return bj_solve(bj, r, z, nullptr, nullptr, nullptr, vec_grid(bj.N * bj.P), s);
}

hipError_t pcg_init(int64_t n, const float* b, const float* M, float floor_, const float* scale, float* x,
                    hipStream_t s, const BlockPrecond* bj) {
    if (bj) return bj_solve(*bj, b, x, nullptr, nullptr, nullptr, vec_grid(n), s);
    hipLaunchKernelGGL(k_init_x, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, b, M, floor_, scale, x);
    return hipGetLastError();
}

hipError_t pcg_init_r(int64_t n, const float* b, const float* g, const float* M, float floor_, const float* scale,
                      float* r, float* z, float* p, double* part, PcgState* st, hipStream_t s,
                      const BlockPrecond* bj) {
    const unsigned nb = vec_grid(n);
    hipLaunchKernelGGL(k_init_r, dim3(nb), dim3(kBlock), 0, s, n, b, g, M, floor_, scale, r, z, p, part);
    if (bj) {   // z0 = A^-1 r0, p0 = z0, and the r.z partials in place of the Jacobi ones
        hipError_t e = bj_solve(*bj, r, z, p, part, nullptr, nb, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(kBlock), 0, s, part, (int64_t)nb, st);
    return hipGetLastError();
}

hipError_t pcg_alpha(const double* pg_part, int64_t nb, PcgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kBlock), 0, s, pg_part, nb, st);
    return hipGetLastError();
}

hipError_t pcg_update(int64_t n, PcgState* st, float* p, const float* g, const float* M, float floor_,
                      const float* scale, float* x, float* r, float* z, double* part, double tol, int tol_mode,
                      hipStream_t s, const BlockPrecond* bj) {
    const unsigned nb = vec_grid(n);
    hipLaunchKernelGGL(k_update_xrz, dim3(nb), dim3(kBlock), 0, s, n, st, p, g, M, floor_, scale, x, r, z, part);
    if (bj) {
        hipError_t e = bj_solve(*bj, r, z, nullptr, part, st, nb, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_beta, dim3(1), dim3(kBlock), 0, s, part, (int64_t)nb, st, tol, tol_mode);
    hipLaunchKernelGGL(k_update_p, dim3(nb), dim3(kBlock), 0, s, n, st, z, p);
    return hipGetLastError();
}

hipError_t launch_combine(int n_b, const float* const* d, const float* const* m, int64_t n, float* out,
                          hipStream_t s) {
    CombineArgs a{};
    a.nb = n_b;
    for (int i = 0; i < n_b; ++i) {
        a.d[i] = d[i];
        a.m[i] = m[i];
    }
    hipLaunchKernelGGL(k_combine, dim3(vec_grid(n)), dim3(kBlock), 0, s, a, n, out);
    return hipGetLastError();
}

}  // namespace lm
