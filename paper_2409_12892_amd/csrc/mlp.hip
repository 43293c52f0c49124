// Learned diagonal preconditioner: an 8 -> 64 -> 64 -> p_out perceptron with
// exact (erf) GELU, evaluated and trained on the matrix cores.  It extends
// the Jacobi preconditioner of Algorithm 1 (section 3.3): the prediction s
// per parameter scales the Jacobi inverse, M^-1 = exp(s) / diag(J^T J).
//
// Every product runs as v_mfma_f32_16x16x16_bf16 in the transposed form
// Y^T = W^T X^T: the output neurons are the rows and 16 samples the columns
// of a 16 x 16 tile.  The accumulator layout of that instruction (lane
// c + 16 (r / 4) holds element (r, c) in register r % 4) is the layout of
// its B operand with the row index as the reduction index, so each layer's
// output, after bias, GELU and rounding to bfloat16, is the next layer's B
// operand without any data movement.  Weights are bfloat16 copies in LDS,
// stored both [out][in] (A operands of the forward products) and [in][out]
// (A operands of the backward products); accumulation is float32.
//
// The weight gradients contract over samples, which are the columns of the
// tiles; a per-wave LDS transpose turns them into the reduction index.  Each
// wave accumulates its gradient over its sample tiles and writes it to a
// partial slot; one pass sums the partials in a fixed order (deterministic)
// and applies Adam.
#include "lm_internal.h"

namespace lm {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kF = 8, kH = 64, kOutMax = 64;
constexpr int oW1 = 0, oB1 = oW1 + kF * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kOutMax;
static_assert(oB3 + kOutMax == kMlpParams, "weight layout");

constexpr int kMlpBlock = 256, kMlpWaves = kMlpBlock / kWave;
constexpr int kLd1 = 20;   // row stride (bf16) of the layer-1 weights, inputs padded 8 -> 16
constexpr int kLd = 68;    // row stride of the 64 x 64 weights (padding spreads the LDS banks)
constexpr int kLdT = 20;   // row stride of the per-wave transpose tiles (16 samples)
constexpr int kMaxParts = 1024;
constexpr float kScaleClamp = 4.0f;   // |s| <= 4: the scale stays within [e^-4, e^4]

__device__ __forceinline__ short bf(float f) { return (short)f32_to_bf16_rne(f); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 lds4(const short* p) { return *reinterpret_cast<const bf16x4*>(p); }

// A zero the compiler cannot see through.  Added to the weight and bias
// addresses inside the sample loop, it keeps their loads in the loop instead
// of hoisting ~180 loop-invariant registers out of it.
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// Orders the LDS accesses of one wave around a wave-private transpose.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct alignas(16) WeightsLds {
    short wt1[kH * kLd1];   // [out][in], in padded with zeros to 16
    short wt2[kH * kLd];    // [out][in]
    short wt3[kH * kLd];    // [out][in]
    short w2[kH * kLd];     // [in][out]
    short w3[kH * kLd];     // [in][out]
};

template <bool BACKWARD>
__device__ void load_weights(const float* __restrict__ w, WeightsLds& L) {
    for (int e = threadIdx.x; e < kH * 16; e += blockDim.x) {
        const int o = e / 16, i = e % 16;
        L.wt1[o * kLd1 + i] = i < kF ? bf(w[oW1 + i * kH + o]) : (short)0;
    }
    for (int e = threadIdx.x; e < kH * kH; e += blockDim.x) {
        const int i = e / kH, o = e % kH;
        const short a = bf(w[oW2 + e]), b = bf(w[oW3 + e]);
        L.wt2[o * kLd + i] = a;
        L.wt3[o * kLd + i] = b;
        if (BACKWARD) {
            L.w2[i * kLd + o] = a;
            L.w3[i * kLd + o] = b;
        }
    }
}

// Bias of the rows this lane holds in output tile t: neurons 16 t + 4 (lane / 16) + r.
__device__ __forceinline__ f32x4 bias4(const float* b, int t, int lg) {
    const float* p = b + 16 * t + 4 * lg;
    return f32x4{p[0], p[1], p[2], p[3]};
}

struct Fwd {
    f32x4 z1[4], z2[4], s[4];
    bf16x4 h1[4], h2[4];
};

// Forward pass of the 16 samples g0 .. g0 + 15 (columns); lane column c = lane % 16.
__device__ __forceinline__ void forward_tile(const WeightsLds& L, const float* __restrict__ w,
                                             const float* __restrict__ feat, int64_t n, int64_t g0, int nt3,
                                             Fwd& F) {
    const int z = opaque_zero();
    const int lane = __lane_id(), lc = lane & 15, lg = (lane >> 4) + z;
    const int64_t g = g0 + lc;
    const bool valid = g < n;
    bf16x4 xb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 4 * lg + q;
        xb[q] = (k < kF && valid) ? bf(feat[(int64_t)k * n + g]) : (short)0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        F.z1[t] = mfma(lds4(&L.wt1[(16 * t + lc) * kLd1 + 4 * lg]), xb, bias4(w + oB1, t, lg));
#pragma unroll
        for (int r = 0; r < 4; ++r) F.h1[t][r] = bf(gelu(F.z1[t][r]));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = bias4(w + oB2, t, lg);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma(lds4(&L.wt2[(16 * t + lc) * kLd + 16 * kk + 4 * lg]), F.h1[kk], acc);
        F.z2[t] = acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) F.h2[t][r] = bf(gelu(acc[r]));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < nt3) {
            f32x4 acc = bias4(w + oB3, t, lg);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = mfma(lds4(&L.wt3[(16 * t + lc) * kLd + 16 * kk + 4 * lg]), F.h2[kk], acc);
            F.s[t] = acc;
        } else {
            F.s[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
}

__global__ void __launch_bounds__(kMlpBlock) k_mlp_forward(const float* __restrict__ w, const float* __restrict__ feat,
                                                          int64_t n, int p_out, float* __restrict__ s_out,
                                                          float* __restrict__ scale_out,
                                                          uint32_t* __restrict__ n_fallback) {
    __shared__ WeightsLds L;
    load_weights<false>(w, L);
    __syncthreads();
    const int lane = __lane_id(), lc = lane & 15, lg = lane >> 4;
    const int nt3 = (p_out + 15) / 16;
    const int64_t n_tiles = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * kMlpWaves + threadIdx.x / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * kMlpWaves;
    uint32_t fallbacks = 0;
    for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
        Fwd F;
        forward_tile(L, w, feat, n, tile * 16, nt3, F);
        const int64_t g = tile * 16 + lc;
        if (g >= n) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= nt3) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * t + 4 * lg + r;
                if (o >= p_out) continue;
                const float s = F.s[t][r];
                const bool ok = isfinite(s);
                fallbacks += ok ? 0u : 1u;
                if (s_out) s_out[(int64_t)o * n + g] = s;
                if (scale_out)
                    scale_out[(int64_t)o * n + g] = ok ? expf(fminf(fmaxf(s, -kScaleClamp), kScaleClamp)) : 1.0f;
            }
        }
    }
    if (n_fallback) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) fallbacks += __shfl_xor(fallbacks, off, kWave);
        if (lane == 0 && fallbacks) atomicAdd(n_fallback, fallbacks);
    }
}

struct alignas(16) TransposeLds {
    short a[kMlpWaves][kH * kLdT];   // rows: output neurons, columns: samples
    short b[kMlpWaves][kH * kLdT];   // rows: input neurons, columns: samples
};

// Stores a D-layout tile (rows 16 t + 4 (lane / 16) + r, column lane % 16) as [row][sample].
__device__ __forceinline__ void put_rows(short* T, int t, f32x4 v, int lc, int lg) {
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * t + 4 * lg + r) * kLdT + lc] = bf(v[r]);
}
__device__ __forceinline__ void put_rows(short* T, int t, bf16x4 v, int lc, int lg) {
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * t + 4 * lg + r) * kLdT + lc] = v[r];
}

// Gradient of sum over (sample, output) of mask (s - target)^2 for the
// samples of this wave, written to the wave's partial slot, with the
// masked squared error and the mask count.
__global__ void __launch_bounds__(kMlpBlock) k_mlp_grad(const float* __restrict__ w, const float* __restrict__ feat,
                                                       const float* __restrict__ target,
                                                       const float* __restrict__ mask, int64_t n, int p_out,
                                                       float* __restrict__ gpart, double* __restrict__ lpart) {
    __shared__ WeightsLds L;
    __shared__ TransposeLds X;
    load_weights<true>(w, L);
    __syncthreads();
    const int lane = __lane_id(), lc = lane & 15, lg = lane >> 4, wid = threadIdx.x / kWave;
    short* TA = X.a[wid];
    short* TB = X.b[wid];
    const int nt3 = (p_out + 15) / 16;
    const int64_t n_tiles = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * kMlpWaves + wid;
    const int64_t n_waves = (int64_t)gridDim.x * kMlpWaves;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    const short one = bf(1.0f);
    const bf16x4 ones = {one, one, one, one};
    // gW*[out tile][in tile] hold the transposed weight gradients; gb* the
    // bias gradients as products with a ones operand (every column holds
    // the sum over samples), so all accumulators stay in MFMA registers
    f32x4 gW3[4][4], gW2[4][4], gW1[4], gb1[4], gb2[4], gb3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gW1[t] = gb1[t] = gb2[t] = gb3[t] = zero;
#pragma unroll
        for (int u = 0; u < 4; ++u) gW3[t][u] = gW2[t][u] = zero;
    }
    double loss = 0.0, cnt = 0.0;
    for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
        const int64_t g0 = tile * 16, g = g0 + lc;
        const int lgz = lg + opaque_zero();
        Fwd F;
        forward_tile(L, w, feat, n, g0, nt3, F);
        // output residual: ds = 2 mask (s - target), zero outside the data
        bf16x4 dsb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * t + 4 * lgz + r;
                const bool v = t < nt3 && o < p_out && g < n;
                const float m = v ? mask[(int64_t)o * n + g] : 0.0f;
                const float tt = v ? target[(int64_t)o * n + g] : 0.0f;
                const float d = m != 0.0f ? (F.s[t][r] - tt) * m : 0.0f;
                loss += (double)d * (double)d;
                cnt += (double)m;
                dsb[t][r] = bf(2.0f * d);
            }
        }
        // gW3^T += ds h2^T (contraction over the 16 samples)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < nt3) put_rows(TA, t, dsb[t], lc, lg);
            put_rows(TB, t, F.h2[t], lc, lg);
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= nt3) continue;
            const bf16x4 a = lds4(&TA[(16 * t + lc) * kLdT + 4 * lg]);
            gb3[t] = mfma(a, ones, gb3[t]);
#pragma unroll
            for (int u = 0; u < 4; ++u) gW3[t][u] = mfma(a, lds4(&TB[(16 * u + lc) * kLdT + 4 * lg]), gW3[t][u]);
        }
        wave_sync();
        // dz2 = (W3 ds) * gelu'(z2)
        bf16x4 dz2b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f32x4 acc = zero;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                if (kk < nt3) acc = mfma(lds4(&L.w3[(16 * u + lc) * kLd + 16 * kk + 4 * lgz]), dsb[kk], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) dz2b[u][r] = bf(acc[r] * gelu_grad(F.z2[u][r]));
        }
        // gW2^T += dz2 h1^T
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            put_rows(TA, t, dz2b[t], lc, lg);
            put_rows(TB, t, F.h1[t], lc, lg);
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x4 a = lds4(&TA[(16 * t + lc) * kLdT + 4 * lg]);
            gb2[t] = mfma(a, ones, gb2[t]);
#pragma unroll
            for (int u = 0; u < 4; ++u) gW2[t][u] = mfma(a, lds4(&TB[(16 * u + lc) * kLdT + 4 * lg]), gW2[t][u]);
        }
        wave_sync();
        // dz1 = (W2 dz2) * gelu'(z1)
        bf16x4 dz1b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f32x4 acc = zero;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = mfma(lds4(&L.w2[(16 * u + lc) * kLd + 16 * kk + 4 * lgz]), dz2b[kk], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) dz1b[u][r] = bf(acc[r] * gelu_grad(F.z1[u][r]));
        }
        // gW1^T += dz1 x^T; the features come straight from memory as [input][sample]
#pragma unroll
        for (int t = 0; t < 4; ++t) put_rows(TA, t, dz1b[t], lc, lg);
        bf16x4 xb;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gs = g0 + 4 * lg + q;
            xb[q] = (lc < kF && gs < n) ? bf(feat[(int64_t)lc * n + gs]) : (short)0;
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x4 a = lds4(&TA[(16 * t + lc) * kLdT + 4 * lg]);
            gW1[t] = mfma(a, xb, gW1[t]);
            gb1[t] = mfma(a, ones, gb1[t]);
        }
        wave_sync();
    }
    // the wave's partial gradient in the weight layout
    float* out = gpart + wave * kMlpParams;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int o = 16 * t + 4 * lg;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = 16 * u + lc;
            *reinterpret_cast<f32x4*>(out + oW3 + i * kH + o) = gW3[t][u];
            *reinterpret_cast<f32x4*>(out + oW2 + i * kH + o) = gW2[t][u];
        }
        if (lc < kF) *reinterpret_cast<f32x4*>(out + oW1 + lc * kH + o) = gW1[t];
        if (lc == 0) {
            *reinterpret_cast<f32x4*>(out + oB1 + o) = gb1[t];
            *reinterpret_cast<f32x4*>(out + oB2 + o) = gb2[t];
            *reinterpret_cast<f32x4*>(out + oB3 + o) = gb3[t];
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        loss += __shfl_xor(loss, off, kWave);
        cnt += __shfl_xor(cnt, off, kWave);
    }
    if (lane == 0) {
        lpart[2 * wave] = loss;
        lpart[2 * wave + 1] = cnt;
    }
}

// Sums the partials in wave order and takes one Adam step (lr > 0):
// m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void __launch_bounds__(kBlock) k_mlp_reduce_adam(const float* __restrict__ gpart,
                                                           const double* __restrict__ lpart, int nparts,
                                                           float* __restrict__ w, float* __restrict__ am,
                                                           float* __restrict__ av, int step, float lr,
                                                           float* __restrict__ grad_out,
                                                           double* __restrict__ loss_out) {
    __shared__ double sh_cnt[kBlock], sh_loss[kBlock];
    double c = 0.0, l = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
        l += lpart[2 * k];
        c += lpart[2 * k + 1];
    }
    sh_cnt[threadIdx.x] = c;
    sh_loss[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double cs = 0.0, ls = 0.0;
        for (int k = 0; k < kBlock; ++k) {
            cs += sh_cnt[k];
            ls += sh_loss[k];
        }
        sh_cnt[0] = cs;
        sh_loss[0] = ls;
    }
    __syncthreads();
    const double cnt = sh_cnt[0];
    const double inv = cnt > 0.0 ? 1.0 / cnt : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) *loss_out = sh_loss[0] * inv;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kMlpParams) return;
    double a = 0.0;
    for (int k = 0; k < nparts; ++k) a += (double)gpart[(int64_t)k * kMlpParams + p];
    const float gr = (float)(a * inv);
    if (grad_out) grad_out[p] = gr;
    if (lr > 0.0f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float m = b1 * am[p] + (1.0f - b1) * gr;
        const float v = b2 * av[p] + (1.0f - b2) * gr * gr;
        am[p] = m;
        av[p] = v;
        const float mh = m / (1.0f - powf(b1, (float)step));
        const float vh = v / (1.0f - powf(b2, (float)step));
        w[p] -= lr * mh / (sqrtf(vh) + eps);
    }
}

unsigned mlp_grid(int64_t n) {
    const int64_t tiles = (n + 15) / 16;
    const int64_t blocks = (tiles + kMlpWaves - 1) / kMlpWaves;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, kMaxParts / kMlpWaves));
}

}  // namespace

int mlp_grad_parts() { return kMaxParts; }

hipError_t launch_mlp_forward(const float* w, const float* feat, int64_t n, int p_out, float* s_out, float* scale_out,
                              uint32_t* n_fallback, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t tiles = (n + 15) / 16;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + kMlpWaves - 1) / kMlpWaves, 2048));
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kMlpBlock), 0, s, w, feat, n, p_out, s_out, scale_out,
                       n_fallback);
    return hipGetLastError();
}

hipError_t launch_mlp_grad_step(float* w, float* adam_m, float* adam_v, int step, float lr, const float* feat,
                                const float* target, const float* mask, int64_t n, int p_out, float* grad_out,
                                double* loss_out, float* gpart, double* lpart, hipStream_t s) {
    const unsigned grid = mlp_grid(n);
    const int nparts = (int)grid * kMlpWaves;
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(kMlpBlock), 0, s, w, feat, target, mask, n, p_out, gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(grid_for(kMlpParams)), dim3(kBlock), 0, s, gpart, lpart, nparts, w,
                       adam_m, adam_v, step, lr, grad_out, loss_out);
    return hipGetLastError();
}

}  // namespace lm
