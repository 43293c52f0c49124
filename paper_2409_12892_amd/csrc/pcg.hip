// Vector half of Algorithm 1 (PCG) with float64 dot products and scalars
// kept on the device, and the subset combination (eq. combine-pcg).
//
// Every kernel of an iteration reads the device `stop` flag first and
// returns when it is set, so the host enqueues n_iters iterations without
// synchronising and the loop still ends where Algorithm 1 breaks.
#include <mutex>

#include "lm_internal.h"

namespace lm {



namespace {

constexpr int kVecBlocks = 2048;   // fixed grid: partial sums in a fixed order


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
// Factors (apply.hip, k_bj_factor): per Gaussian the packed lower Cholesky
// factor of its damped block, element t = i (i + 1) / 2 + j (the diagonal
// slot holding 1 / L_ii), stored in tiles of 64 Gaussians,
// L[g / 64][t][g % 64]: a wave's 64 Gaussians read one contiguous tile.

// z = A^-1 r, one thread per Gaussian over a fixed grid (the PCG partial
// grid): forward substitution L y = r, then backward L^T z = y, both
// walking the factor row by row (coalesced across the wave's Gaussians;
// the factor is read twice).  The thread's vector lives in LDS, one column
// per thread (conflict-free).  Writes z (and a copy to z2 when given) and
// the block partials of r . z.
template <int P>
__global__ void __launch_bounds__(kBlock) k_bj_solve(const float* __restrict__ L, int64_t N,
                                                   const float* __restrict__ r, float* __restrict__ z,
                                                   float* __restrict__ z2, double* __restrict__ part,
                                                   const PcgState* __restrict__ st) {
    if (st && st->stop) return;
    __shared__ float sy[P][kBlock];
    float* y = &sy[0][threadIdx.x];
    double acc[1] = {0.0};
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < N; g += (int64_t)gridDim.x * kBlock) {
#pragma unroll 1
        for (int i = 0; i < P; ++i) y[i * kBlock] = r[(int64_t)i * N + g];
        constexpr int T = P * (P + 1) / 2;
        const float* Lt = L + (g >> 6) * (int64_t)T * 64 + (g & 63);
        const float* Lp = Lt;
#pragma unroll 1
        for (int i = 0; i < P; ++i) {
            float v = y[i * kBlock];
#pragma unroll 8
            for (int j = 0; j < i; ++j) {
                v -= *Lp * y[j * kBlock];
                Lp += 64;
            }
            y[i * kBlock] = v * *Lp;
            Lp += 64;
        }
#pragma unroll 1
        for (int i = P - 1; i >= 0; --i) {
            const float* Lr = Lt + (int64_t)(i * (i + 1) / 2) * 64;
            const float zi = y[i * kBlock] * Lr[i * 64];
            y[i * kBlock] = zi;
#pragma unroll 8
            for (int j = 0; j < i; ++j) {
                y[j * kBlock] -= *Lr * zi;
                Lr += 64;
            }
        }
#pragma unroll 1
        for (int i = 0; i < P; ++i) {
            const float zi = y[i * kBlock];
            z[(int64_t)i * N + g] = zi;
            if (z2) z2[(int64_t)i * N + g] = zi;
            acc[0] += (double)r[(int64_t)i * N + g] * zi;
        }
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

// float64 dot product of two float32 vectors: per-block partial sums over a
// fixed grid, then one block sums them (fixed order, deterministic)
__global__ void k_dot_part(int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                           double* __restrict__ part) {
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[0] += (double)a[i] * (double)b[i];
    block_partials<1>(v, part, 0);
}

__global__ void k_dot_sum(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
    const double r = block_sum(part, nb);
    if (threadIdx.x == 0) *out = r;
}

__global__ void k_axpy(int64_t n, const float* __restrict__ x, const float* __restrict__ d, float gamma,
                       float* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = fmaf(gamma, d[i], x[i]);
}

}  // namespace

int64_t pcg_partial_count(int64_t n) { return vec_grid(n); }

int64_t dot_partial_count(int64_t n) { return vec_grid(n); }

hipError_t launch_dot(const float* a, const float* b, int64_t n, double* part, double* out, hipStream_t s) {
    const unsigned nb = vec_grid(n);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(kBlock), 0, s, n, a, b, part);
    hipLaunchKernelGGL(k_dot_sum, dim3(1), dim3(kBlock), 0, s, part, (int64_t)nb, out);
    return hipGetLastError();
}

// Partial sums of lm_vec_dot_static: a library-owned device array, one
// copy per GPU (a __device__ variable lives in every device's copy of the
// code object), sized for the fixed vector grid.  Host code never passes
// the array's name to a kernel (on the host it is a stand-in, not a device
// address); the address is looked up once per device, with that device
// current, and used for every later call on it.
static __device__ __align__(256) double scratch[kVecBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];
}  // namespace

int64_t dot_static_capacity() { return kVecBlocks; }

hipError_t dot_static_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

hipError_t launch_axpy(const float* x, const float* d, float gamma, int64_t n, float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, x, d, gamma, out);
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
