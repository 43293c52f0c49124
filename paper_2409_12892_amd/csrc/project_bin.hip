// Projection of every (Gaussian, view) in float64 and tile binning.
//
// Binning is an integer function of float32 records: mean and depth are the
// float64 projection rounded to float32, the tile rectangle is
// floor((m -/+ r) / tile) evaluated in float32 (IEEE division) with inclusive
// bounds, and the sort key is (global tile index << 31) | float32 depth bits
// (depth > 0.2, so its sign bit is zero).  Values are Gaussian ids emitted in
// id order per view, so the stable radix sort breaks depth ties by id.
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

// rec64 layout [10][V*N]: mx, my, A, B, C, o, log threshold, r, g, b (float64)
template <int deg>
__global__ void k_project(const CamDev* __restrict__ cams, const float* __restrict__ x, int64_t N, int V,
                          int TW, int TH, double* __restrict__ rec64, float* __restrict__ recf,
                          int32_t* __restrict__ rad, uint32_t* __restrict__ keycnt) {
    const int64_t R = N * (int64_t)V;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
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
    for (int i = 0; i < 10; ++i) rec64[(int64_t)i * R + r] = vals[i];
}

__global__ void k_bin_emit(const CamDev* __restrict__ cams, int64_t N, int V, int TW, int TH,
                           const float* __restrict__ recf, const int32_t* __restrict__ rad,
                           const uint32_t* __restrict__ keycnt, const uint64_t* __restrict__ keyoff,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t R = N * (int64_t)V;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R || keycnt[r] == 0) return;
    const int v = (int)(r / N);
    const uint32_t g = (uint32_t)(r - (int64_t)v * N);
    const CamDev& cam = cams[v];
    int x0, y0, x1, y1;
    tile_rect(recf[r], recf[R + r], rad[r], TW, TH, cam.TX, cam.TY, x0, y0, x1, y1);
    const uint64_t zbits = (uint64_t)__float_as_uint(recf[2 * R + r]);
    uint64_t o = keyoff[r];
    for (int ty = y0; ty <= y1; ++ty)
        for (int tx = x0; tx <= x1; ++tx) {
            const uint64_t tile = (uint64_t)(cam.tile_base + (int64_t)ty * cam.TX + tx);
            keys[o] = (tile << 31) | zbits;
            vals[o] = g;
            ++o;
        }
}

// tile_start[t] = first key index of tile t (lists are [tile_start[t], tile_start[t+1])).
__global__ void k_tile_ranges(const uint64_t* __restrict__ keys, int64_t K, int64_t n_tiles,
                              int64_t* __restrict__ tile_start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const int64_t t = (int64_t)(keys[i] >> 31);
    const int64_t tp = i == 0 ? -1 : (int64_t)(keys[i - 1] >> 31);
    for (int64_t u = tp + 1; u <= t; ++u) tile_start[u] = i;
    if (i == K - 1)
        for (int64_t u = t + 1; u <= n_tiles; ++u) tile_start[u] = K;
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

hipError_t launch_bin_emit(const CamDev* cams, int64_t N, int V, int TW, int TH, const float* recf,
                           const int32_t* rad, const uint32_t* keycnt, const uint64_t* keyoff, uint64_t* keys,
                           uint32_t* vals, hipStream_t s) {
    const int64_t R = N * (int64_t)V;
    hipLaunchKernelGGL(k_bin_emit, dim3(grid_for(R)), dim3(kBlock), 0, s, cams, N, V, TW, TH, recf, rad, keycnt,
                       keyoff, keys, vals);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint64_t* keys, int64_t K, int64_t n_tiles, int64_t* tile_start,
                              hipStream_t s) {
    if (K == 0) {
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n_tiles + 1)), dim3(kBlock), 0, s, tile_start, n_tiles + 1,
                           (int64_t)0);
    } else {
        hipLaunchKernelGGL(k_tile_ranges, dim3(grid_for(K)), dim3(kBlock), 0, s, keys, K, n_tiles, tile_start);
    }
    return hipGetLastError();
}

}  // namespace lm
