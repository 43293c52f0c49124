// Float64 projection of one Gaussian into one view (the "ds/dx" factor of
// paper eq. backward-pass) and its forward-mode tangent.  The paper defers the projection to the original 3DGS rasteriser
// (EWA splatting); the conventions here are: quaternion (w,x,y,z) normalised
// before use, Sigma = R diag(exp(2 s)) R^T, t = R_v mu + t_v, pinhole mean
// m = f t_xy / t_z + c, screen covariance J W J^T + 0.3 I with the
// perspective Jacobian J at t, conic = inverse screen covariance, opacity =
// sigmoid(logit), colour = max(0, 0.5 + sum_k Y_k(d) f_k) with the real SH
// basis at the unit view direction d = (mu - C_v) / |mu - C_v|.
//
// The splat attributes are y = (m_x, m_y, A, B, C, o, r, g, b) and the pixel
// exponent is -0.5 (A dx^2 + C dy^2) - B dx dy with d = pixel - m.
//
// Tangents are handed to the pair kernels in the "power coefficient" form
// (P1, P2, Q1, Q2, Q3, do, dr, dg, db): for a pixel offset d,
//     d alpha = alpha (P1 dx + P2 dy + Q1 dx^2 + Q2 dx dy + Q3 dy^2) + G do
// with P1 = A dm_x + B dm_y, P2 = B dm_x + C dm_y, Q1 = -dA/2, Q2 = -dB,
// Q3 = -dC/2 (G = exp(power)).
#pragma once

#include "lm_internal.h"

namespace lm {

// Real spherical harmonics, degrees 0..3, index k = l*l + l + m.
namespace shc {
constexpr double C0 = 0.28209479177387814;
constexpr double C1 = 0.4886025119029199;
constexpr double C2a = 1.0925484305920792, C2b = 0.31539156525252005, C2c = 0.5462742152960396;
constexpr double C3a = 0.5900435899266435, C3b = 2.890611442640554, C3c = 0.4570457994644658;
constexpr double C3d = 0.3731763325901154, C3e = 1.445305721320277;
}  // namespace shc

template <int deg>
__device__ __forceinline__ void sh_eval(const double d[3], double Y[16]) {
    using namespace shc;
    const double x = d[0], y = d[1], z = d[2];
    Y[0] = C0;
    if constexpr (deg < 1) return;
    Y[1] = C1 * y; Y[2] = C1 * z; Y[3] = C1 * x;
    if constexpr (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = C2a * x * y;
    Y[5] = C2a * y * z;
    Y[6] = C2b * (2.0 * zz - xx - yy);
    Y[7] = C2a * x * z;
    Y[8] = C2c * (xx - yy);
    if constexpr (deg < 3) return;
    Y[9] = C3a * y * (3.0 * xx - yy);
    Y[10] = C3b * x * y * z;
    Y[11] = C3c * y * (4.0 * zz - xx - yy);
    Y[12] = C3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = C3c * x * (4.0 * zz - xx - yy);
    Y[14] = C3e * z * (xx - yy);
    Y[15] = C3a * x * (xx - 3.0 * yy);
}

// dY[k] = grad Y_k(d) . v  (gradients of the polynomials above in R^3)
template <int deg>
__device__ __forceinline__ void sh_grad_dot(const double d[3], const double v[3], double dY[16]) {
    using namespace shc;
    const double x = d[0], y = d[1], z = d[2];
    const double vx = v[0], vy = v[1], vz = v[2];
    dY[0] = 0.0;
    if constexpr (deg < 1) return;
    dY[1] = C1 * vy; dY[2] = C1 * vz; dY[3] = C1 * vx;
    if constexpr (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    dY[4] = C2a * (y * vx + x * vy);
    dY[5] = C2a * (z * vy + y * vz);
    dY[6] = C2b * (-2.0 * x * vx - 2.0 * y * vy + 4.0 * z * vz);
    dY[7] = C2a * (z * vx + x * vz);
    dY[8] = C2c * (2.0 * x * vx - 2.0 * y * vy);
    if constexpr (deg < 3) return;
    dY[9] = C3a * (6.0 * x * y * vx + (3.0 * xx - 3.0 * yy) * vy);
    dY[10] = C3b * (y * z * vx + x * z * vy + x * y * vz);
    dY[11] = C3c * (-2.0 * x * y * vx + (4.0 * zz - xx - 3.0 * yy) * vy + 8.0 * y * z * vz);
    dY[12] = C3d * (-6.0 * x * z * vx - 6.0 * y * z * vy + (6.0 * zz - 3.0 * xx - 3.0 * yy) * vz);
    dY[13] = C3c * ((4.0 * zz - 3.0 * xx - yy) * vx - 2.0 * x * y * vy + 8.0 * x * z * vz);
    dY[14] = C3e * (2.0 * x * z * vx - 2.0 * y * z * vy + (xx - yy) * vz);
    dY[15] = C3a * ((3.0 * xx - 3.0 * yy) * vx - 6.0 * x * y * vy);
}

// Partial derivatives of the rotation matrix (row-major) with respect to the
// normalised quaternion components w, x, y, z.
__device__ __forceinline__ void rot_partials(const double q[4], double dR[4][9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double a[4][9] = {
        {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0},
    };
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < 9; ++i) dR[c][i] = a[c][i];
}

struct ProjFwd {
    double mx, my, A, B, C, o, col[3], z;
    int32_t radius;
    bool vis;
    bool clamp[3];
    double t[3], qn[4], qnorm, Rq[9], S[3], M[9], Wc[9], J[6], T2[6], det;
    double d[3], dn, Y[16];
};

// x is the SoA parameter array [P][N]; g the Gaussian index.
template <int deg>
__device__ inline void proj_forward(const CamDev& cam, const float* __restrict__ x, int64_t N, int64_t g,
                                    ProjFwd& f) {
    double mu[3], s[3], q[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) mu[i] = (double)x[(int64_t)i * N + g];
#pragma unroll
    for (int i = 0; i < 3; ++i) s[i] = (double)x[(int64_t)(3 + i) * N + g];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = (double)x[(int64_t)(6 + i) * N + g];
    const double om = (double)x[(int64_t)10 * N + g];
    const double* R = cam.R;
#pragma unroll
    for (int i = 0; i < 3; ++i) f.t[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + cam.t[i];
    const double tz = f.t[2];
    f.z = tz;
    f.vis = tz > kNear;
    f.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) f.qn[i] = q[i] / f.qnorm;
    {
        const double w = f.qn[0], a = f.qn[1], b = f.qn[2], c = f.qn[3];
        f.Rq[0] = 1 - 2 * (b * b + c * c); f.Rq[1] = 2 * (a * b - w * c); f.Rq[2] = 2 * (a * c + w * b);
        f.Rq[3] = 2 * (a * b + w * c); f.Rq[4] = 1 - 2 * (a * a + c * c); f.Rq[5] = 2 * (b * c - w * a);
        f.Rq[6] = 2 * (a * c - w * b); f.Rq[7] = 2 * (b * c + w * a); f.Rq[8] = 1 - 2 * (a * a + b * b);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) f.S[j] = exp(s[j]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) f.M[3 * i + j] = f.Rq[3 * i + j] * f.S[j];
    // world covariance Sigma = M M^T, then camera frame W = R_v Sigma R_v^T
    double Sg[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Sg[3 * i + j] = f.M[3 * i] * f.M[3 * j] + f.M[3 * i + 1] * f.M[3 * j + 1] + f.M[3 * i + 2] * f.M[3 * j + 2];
    double RS[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            RS[3 * i + j] = R[3 * i] * Sg[j] + R[3 * i + 1] * Sg[3 + j] + R[3 * i + 2] * Sg[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            f.Wc[3 * i + j] = RS[3 * i] * R[3 * j] + RS[3 * i + 1] * R[3 * j + 1] + RS[3 * i + 2] * R[3 * j + 2];
    const double fx = cam.fx, fy = cam.fy;
    f.J[0] = fx / tz; f.J[1] = 0.0; f.J[2] = -fx * f.t[0] / (tz * tz);
    f.J[3] = 0.0; f.J[4] = fy / tz; f.J[5] = -fy * f.t[1] / (tz * tz);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            f.T2[3 * i + j] = f.J[3 * i] * f.Wc[j] + f.J[3 * i + 1] * f.Wc[3 + j] + f.J[3 * i + 2] * f.Wc[6 + j];
    const double a = f.T2[0] * f.J[0] + f.T2[1] * f.J[1] + f.T2[2] * f.J[2] + kDilation;
    const double b = f.T2[0] * f.J[3] + f.T2[1] * f.J[4] + f.T2[2] * f.J[5];
    const double c = f.T2[3] * f.J[3] + f.T2[4] * f.J[4] + f.T2[5] * f.J[5] + kDilation;
    f.det = a * c - b * b;
    f.vis = f.vis && f.det > 0.0;
    f.A = c / f.det;
    f.B = -b / f.det;
    f.C = a / f.det;
    f.mx = fx * f.t[0] / tz + cam.cx;
    f.my = fy * f.t[1] / tz + cam.cy;
    const double lam = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b);
    f.radius = (int32_t)ceil(3.0 * sqrt(lam));
    f.o = 1.0 / (1.0 + exp(-om));
    double dv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dv[i] = mu[i] - cam.C[i];
    f.dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) f.d[i] = dv[i] / f.dn;
    sh_eval<deg>(f.d, f.Y);
    constexpr int K = (deg + 1) * (deg + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += f.Y[k] * (double)x[(int64_t)(11 + 3 * k + ch) * N + g];
        f.clamp[ch] = acc < 0.0;
        f.col[ch] = f.clamp[ch] ? 0.0 : acc;
    }
}

// Forward-mode derivative of y along the parameter tangent (dgeo = d mean,
// d log-scale, d quaternion, d opacity logit; dsh = tangent SoA array or
// nullptr).  Writes the power-coefficient form described at the top.
template <int deg>
__device__ inline void proj_tangent(const CamDev& cam, const ProjFwd& f, const double dgeo[11],
                                    const float* __restrict__ x, const float* __restrict__ dsh, int64_t N,
                                    int64_t g, double out[9]) {
    const double* R = cam.R;
    const double fx = cam.fx, fy = cam.fy, tz = f.t[2];
    double dt[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dt[i] = R[3 * i] * dgeo[0] + R[3 * i + 1] * dgeo[1] + R[3 * i + 2] * dgeo[2];
    const double iz2 = 1.0 / (tz * tz);
    const double dmx = fx * (dt[0] * tz - f.t[0] * dt[2]) * iz2;
    const double dmy = fy * (dt[1] * tz - f.t[1] * dt[2]) * iz2;
    // quaternion normalisation and rotation
    const double qd = f.qn[0] * dgeo[6] + f.qn[1] * dgeo[7] + f.qn[2] * dgeo[8] + f.qn[3] * dgeo[9];
    double dqn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dqn[c] = (dgeo[6 + c] - f.qn[c] * qd) / f.qnorm;
    double dRp[4][9];
    rot_partials(f.qn, dRp);
    double dR[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) dR[i] = dRp[0][i] * dqn[0] + dRp[1][i] * dqn[1] + dRp[2][i] * dqn[2] + dRp[3][i] * dqn[3];
    double dM[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dM[3 * i + j] = dR[3 * i + j] * f.S[j] + f.Rq[3 * i + j] * f.S[j] * dgeo[3 + j];
    double dS[9];   // dSigma = dM M^T + M dM^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) v += dM[3 * i + k] * f.M[3 * j + k] + f.M[3 * i + k] * dM[3 * j + k];
            dS[3 * i + j] = v;
        }
    double RS[9], dW[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            RS[3 * i + j] = R[3 * i] * dS[j] + R[3 * i + 1] * dS[3 + j] + R[3 * i + 2] * dS[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dW[3 * i + j] = RS[3 * i] * R[3 * j] + RS[3 * i + 1] * R[3 * j + 1] + RS[3 * i + 2] * R[3 * j + 2];
    double dJ[6] = {-fx * dt[2] * iz2, 0.0, -fx * (dt[0] * iz2 - 2.0 * f.t[0] * dt[2] * iz2 / tz),
                    0.0, -fy * dt[2] * iz2, -fy * (dt[1] * iz2 - 2.0 * f.t[1] * dt[2] * iz2 / tz)};
    // dcov = dJ T2^T + J dW J^T + T2 dJ^T
    double JdW[6];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            JdW[3 * i + j] = f.J[3 * i] * dW[j] + f.J[3 * i + 1] * dW[3 + j] + f.J[3 * i + 2] * dW[6 + j];
    double dc[4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                v += dJ[3 * i + k] * f.T2[3 * j + k] + JdW[3 * i + k] * f.J[3 * j + k] + f.T2[3 * i + k] * dJ[3 * j + k];
            dc[2 * i + j] = v;
        }
    // dK = -K dcov K
    const double K[4] = {f.A, f.B, f.B, f.C};
    double X[4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) X[2 * i + j] = K[2 * i] * dc[j] + K[2 * i + 1] * dc[2 + j];
    const double dA = -(X[0] * K[0] + X[1] * K[2]);
    const double dB = -(X[0] * K[1] + X[1] * K[3]);
    const double dC = -(X[2] * K[1] + X[3] * K[3]);
    const double dop = f.o * (1.0 - f.o) * dgeo[10];
    out[0] = f.A * dmx + f.B * dmy;
    out[1] = f.B * dmx + f.C * dmy;
    out[2] = -0.5 * dA;
    out[3] = -dB;
    out[4] = -0.5 * dC;
    out[5] = dop;
    // colour: direction tangent plus SH coefficient tangent
    double dd[3];
    {
        const double dm0 = dgeo[0], dm1 = dgeo[1], dm2 = dgeo[2];
        const double pr = f.d[0] * dm0 + f.d[1] * dm1 + f.d[2] * dm2;
        dd[0] = (dm0 - f.d[0] * pr) / f.dn;
        dd[1] = (dm1 - f.d[1] * pr) / f.dn;
        dd[2] = (dm2 - f.d[2] * pr) / f.dn;
    }
    double dY[16];
    sh_grad_dot<deg>(f.d, dd, dY);
    constexpr int Kc = (deg + 1) * (deg + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        double v = 0.0;
        if (!f.clamp[ch]) {
#pragma unroll
            for (int k = 0; k < Kc; ++k) {
                const int64_t row = (int64_t)(11 + 3 * k + ch) * N + g;
                v += dY[k] * (double)x[row];
                if (dsh) v += f.Y[k] * (double)dsh[row];
            }
        }
        out[6 + ch] = v;
    }
}

}  // namespace lm
