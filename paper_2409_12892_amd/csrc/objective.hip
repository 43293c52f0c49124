// Residual terms of the rendering objective per pixel and colour channel.
//
// Section 3.1 (eq. sgd-loss, eq. gn-loss): the objective has, per pixel and
// channel, the residuals r1 = sqrt(f1), f1 = lam1 |c - C|, and
// r2 = sqrt(f2), f2 = lam2 (1 - SSIM(c, C)); E = sum f1 + f2.  Supplement
// A.4 (eq. res-sq-root-weights, res-sq-root-weights-sum) splits every
// Jacobian row into dr/dc times the colour Jacobian, so the products need
// two images per view:
//   e = sum_t r_t dr_t/dc = sum_t f_t' / 2          (b = -J^T e)
//   w = sum_t (dr_t/dc)^2 = sum_t f_t'^2 / (4 max(f_t, eps))
// SSIM per channel over an 11 x 11 Gaussian window (sigma 1.5, weights
// summing to 1, pixels outside the image are 0), C1 = 0.01^2, C2 = 0.03^2;
// its derivative goes to the window's centre pixel only (section 3.3).
// For the plain least-squares objective: e = c - C, w = 1, E = sum e^2.
//
// One workgroup per 16 x 16 pixels of one channel of one view: the
// 26 x 26 neighbourhood of both images goes to LDS in float64, the five
// window sums (x, y, xx, yy, xy) are formed separably (rows, then columns),
// and every term is evaluated in float64; w and e are stored as float32.
// E is summed per workgroup and the partials reduced in a fixed order.
#include "lm_internal.h"

namespace lm {
namespace {

constexpr int kOT = 16;              // output tile edge
constexpr int kWinR = 5;             // window radius
constexpr int kWin = 2 * kWinR + 1;
constexpr int kIn = kOT + 2 * kWinR; // staged edge (26)
constexpr double kC1 = 0.01 * 0.01, kC2 = 0.03 * 0.03;

__global__ void __launch_bounds__(kOT * kOT) k_objective(ObjectiveArgs A) {
    __shared__ double sx[kIn][kIn + 1], sy[kIn][kIn + 1];
    __shared__ double hs[5][kIn][kOT];
    __shared__ double red[kOT * kOT / kWave];
    const int tid = threadIdx.x;
    const int ch = blockIdx.z;
    const int W = A.W, H = A.H;
    const int64_t base = A.off + (int64_t)ch * W * H;
    const int lx = tid % kOT, ly = tid / kOT;
    const int px = blockIdx.x * kOT + lx, py = blockIdx.y * kOT + ly;
    const bool valid = px < W && py < H;
    double Ev = 0.0;
    if (A.kind == LM_OBJ_L2) {
        if (valid) {
            const int64_t k = base + (int64_t)py * W + px;
            const double r = A.add_target ? (double)A.a[k] : (double)A.a[k] - (double)A.t[k];
            Ev = r * r;
            if (A.e) A.e[k] = (float)r;
            if (A.w) A.w[k] = 1.0f;
        }
    } else {
        const int x0 = blockIdx.x * kOT - kWinR, y0 = blockIdx.y * kOT - kWinR;
        for (int i = tid; i < kIn * kIn; i += kOT * kOT) {
            const int r = i / kIn, c = i % kIn;
            const int gx = x0 + c, gy = y0 + r;
            double xv = 0.0, yv = 0.0;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const int64_t k = base + (int64_t)gy * W + gx;
                yv = (double)A.t[k];
                xv = A.add_target ? (double)A.a[k] + yv : (double)A.a[k];
            }
            sx[r][c] = xv;
            sy[r][c] = yv;
        }
        __syncthreads();
        for (int i = tid; i < kIn * kOT; i += kOT * kOT) {
            const int r = i / kOT, c = i % kOT;
            double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double g = A.g[k], xv = sx[r][c + k], yv = sy[r][c + k];
                m0 += g * xv;
                m1 += g * yv;
                m2 += g * (xv * xv);
                m3 += g * (yv * yv);
                m4 += g * (xv * yv);
            }
            hs[0][r][c] = m0;
            hs[1][r][c] = m1;
            hs[2][r][c] = m2;
            hs[3][r][c] = m3;
            hs[4][r][c] = m4;
        }
        __syncthreads();
        if (valid) {
            double mx = 0.0, my = 0.0, exx = 0.0, eyy = 0.0, exy = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double g = A.g[k];
                mx += g * hs[0][ly + k][lx];
                my += g * hs[1][ly + k][lx];
                exx += g * hs[2][ly + k][lx];
                eyy += g * hs[3][ly + k][lx];
                exy += g * hs[4][ly + k][lx];
            }
            const double xc = sx[ly + kWinR][lx + kWinR], yc = sy[ly + kWinR][lx + kWinR];
            const double g0 = A.g[kWinR] * A.g[kWinR];
            const double vxx = exx - mx * mx, vyy = eyy - my * my, vxy = exy - mx * my;
            const double Aa = 2.0 * mx * my + kC1, Bb = 2.0 * vxy + kC2;
            const double Cc = mx * mx + my * my + kC1, Dd = vxx + vyy + kC2;
            const double S = (Aa * Bb) / (Cc * Dd);
            const double dA = 2.0 * g0 * my, dB = 2.0 * g0 * (yc - my);
            const double dC = 2.0 * g0 * mx, dD = 2.0 * g0 * (xc - mx);
            const double dS = (dA * Bb + Aa * dB) / (Cc * Dd) - S * (dC * Dd + Cc * dD) / (Cc * Dd);
            const double diff = xc - yc;
            const double f1 = A.lam1 * fabs(diff);
            const double d1 = diff > 0.0 ? A.lam1 : (diff < 0.0 ? -A.lam1 : 0.0);
            const double f2 = fmax(A.lam2 * (1.0 - S), 0.0);
            const double d2 = -A.lam2 * dS;
            Ev = f1 + f2;
            const int64_t k = base + (int64_t)py * W + px;
            if (A.e) A.e[k] = (float)(0.5 * (d1 + d2));
            if (A.w) A.w[k] = (float)(d1 * d1 / (4.0 * fmax(f1, A.eps)) + d2 * d2 / (4.0 * fmax(f2, A.eps)));
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) Ev += __shfl_xor(Ev, off, kWave);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = Ev;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int i = 0; i < kOT * kOT / kWave; ++i) tot += red[i];
        A.part[A.part0 + ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
    }
}

// E per view: workgroup v sums the partials of view v (the views' partial
// ranges follow each other in view order).
__global__ void __launch_bounds__(kBlock) k_objective_view_sums(const CamDev* __restrict__ cams, int V,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ out) {
    __shared__ double sh[kBlock];
    const int v = blockIdx.x;
    int64_t p0 = 0;
    for (int u = 0; u < v; ++u)
        p0 += (int64_t)((cams[u].W + kOT - 1) / kOT) * ((cams[u].H + kOT - 1) / kOT) * 3;
    const int64_t n = (int64_t)((cams[v].W + kOT - 1) / kOT) * ((cams[v].H + kOT - 1) / kOT) * 3;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += part[p0 + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = sh[0];
}

}  // namespace

hipError_t launch_objective_view_sums(const CamDev* cams, int V, const double* part, double* out, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_objective_view_sums, dim3((unsigned)V), dim3(kBlock), 0, s, cams, V, part, out);
    return hipGetLastError();
}

int64_t objective_blocks(int W, int H) {
    return (int64_t)((W + kOT - 1) / kOT) * ((H + kOT - 1) / kOT) * 3;
}

void objective_window(double* g) {
    double s = 0.0;
    for (int k = 0; k < kWin; ++k) {
        const double d = k - kWinR;
        g[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < kWin; ++k) g[k] /= s;
}

hipError_t launch_objective(const ObjectiveArgs& a, hipStream_t s) {
    if (a.W <= 0 || a.H <= 0) return hipSuccess;
    const dim3 g((unsigned)((a.W + kOT - 1) / kOT), (unsigned)((a.H + kOT - 1) / kOT), 3);
    hipLaunchKernelGGL(k_objective, g, dim3(kOT * kOT), 0, s, a);
    return hipGetLastError();
}

}  // namespace lm
