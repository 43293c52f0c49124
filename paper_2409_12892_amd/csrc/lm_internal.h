// Internal definitions shared by the HIP translation units of liblm3dgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lm3dgs.h"

namespace lm {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kMaxTilePix = 256;   // pixels per tile (pixel-in-tile index is one byte)
constexpr int kTileBlocks = 4;     // pixel blocks per tile (the pixels of one raster wave each)
constexpr int kBlockPix = 64;      // pixels per block
constexpr int kWindow = 512;       // pairs (64 runs of 8) a wave takes at a time in the pair passes
constexpr int MODE_J = 1, MODE_JT = 2, MODE_JTJ = 3;   // product pass: J p, J^T u, fused J^T J p
constexpr int kMaxViews = 4096;

// Blending constants (paper section 3.1 defers them to the original 3DGS
// rasteriser): alpha threshold, alpha clamp, transmittance cut-off, near
// plane, screen-space dilation.
constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;
constexpr double kNear = 0.2;
constexpr double kDilation = 0.3;

// Flag bits stored in the cached transmittance word (T in [1e-4, 1], so the
// sign bit and the top exponent bit of its float32/bf16/fp16 encoding are
// always zero and carry per-pair flags instead).
constexpr uint32_t kHeadBit32 = 0x80000000u, kClampBit32 = 0x40000000u;
constexpr uint16_t kHeadBit16 = 0x8000u, kClampBit16 = 0x4000u;

// Camera in float64 plus its place in the subset's pixel and tile arrays.
struct CamDev {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double C[3];          // camera centre in world coordinates, -R^T t
    int32_t W, H, TX, TY;
    int64_t tile_base;    // first global tile index of this view
    int64_t pix_base;     // first global pixel index (v-major, then row, column)
};

// Everything a kernel needs to read the cache of one subset.
struct CacheView {
    int64_t N;
    int32_t P, deg, V, TW, TH, dtype;
    int32_t tw_shift;            // log2(TW); tile widths are powers of two
    int64_t n_tiles, n_pix, n_seg, n_gv;
    const CamDev* cams;          // dev [V]
    const int32_t* tile_view;    // dev [n_tiles] view of each tile
    const int64_t* tile_pair_off;// dev [n_tiles+1]
    const int64_t* tile_seg_off; // dev [n_tiles+1]
    const void* pT;              // dev [n_pairs] cache words (float or 16-bit)
    const void* pD;              // dev [3][pair_stride]
    const uint8_t* ppix;         // dev [n_pairs] pixel-in-tile index
    int64_t n_pairs;             // pair slots including the zero padding of each segment to 8
    int64_t pair_stride;         // plane stride of pT/pD/ppix (>= n_pairs + 8, multiple of 8)
    const uint32_t* seg_gv;      // dev [n_seg] active (Gaussian, view) index
    const uint32_t* tile_blk;    // dev [n_tiles][4] padded pairs of each pixel block (blocks in order)
    const float* seg_f;          // dev [6][seg_stride]: mean-in-tile x, y, A, B, C, opacity
    int64_t seg_stride;
    const uint32_t* run_seg;     // dev [pair_stride / 8]: segment of each aligned 8-pair run
    const uint32_t* gv_rec;      // dev [n_gv] record index v*N + g
    const uint32_t* gv_first;    // dev [N+1] first gv of each Gaussian
    const uint32_t* gv_seg_off;  // dev [n_gv+1]
    const uint32_t* gv_segs;     // dev [n_seg] segment ids grouped by gv, ascending
    const uint32_t* seg_pos;     // dev [n_seg] position of each segment in gv_segs
    const uint32_t* list_gv;     // dev [n_seg] gv of each gv_segs entry
    const float* lin;            // dev [kLin][lin_stride]: linearised projection per gv
    int64_t lin_stride;
    const float* wres;           // dev [3 * n_pix] residual weights (image layout), or null: all 1
    // thinned cache (thin_k = K > 0): tile_pair_off and tile_blk count
    // pieces (a splat's pixels in one 64-pixel block), seg_f has 9 rows
    // (+ colour), and there are no pair planes
    int32_t thin_k;
    const uint32_t* piece_seg;   // dev [n_pieces] segment of each piece
    const uint64_t* piece_mask;  // dev [n_pieces] contributing pixels (lane bits of the block)
    const uint64_t* piece_cmask; // dev [n_pieces] those whose alpha is clamped
    const int64_t* tile_ck_off;  // dev [n_tiles + 1] first checkpoint of each tile
    const uint32_t* pix_ck;      // dev [n_pix] first checkpoint of each pixel within its tile's range
    const float4* ck;            // dev [n_ck + 2] T, S0, S1, S2 in front of every K-th contributor
};

// Linearisation of the projection of one (Gaussian, view) at the cache's x,
// stored per gv (float32, index k of lin[k * lin_stride + gv]):
//   L[i][j]     k = i*11 + j        d a_i / d xgeo_j, a = (P1, P2, Q1, Q2, Q3, do)
//                                   (power-coefficient form), xgeo = mean,
//                                   log-scale, quaternion, opacity logit
//   Jdir[ch][m] k = 66 + 3 ch + m   d colour_ch / d mean_m through the view
//                                   direction (0 for a clamped channel)
//   Y[k]        k = 75 + k          SH basis at the view direction
//   mask[ch]    k = 91 + ch         1, or 0 for a clamped channel
constexpr int kLinL = 0, kLinJdir = 66, kLinY = 75, kLinMask = 91, kLin = 94;

// Thread-local error message plumbing.
void set_error(const std::string& msg);
#define LM_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::lm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
            return LM_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

// Blocks of one thread per element.  A launch's work-item count is a 32-bit
// number: kernels whose element count can reach 2^32 (the tile keys of a
// large subset) loop grid-stride over a capped grid instead.
inline unsigned grid_for(int64_t n, int block = kBlock) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// M^-1 of Algorithm 1 with the optional minimum diagonal (0 where M = 0) and
// an optional learned scale per parameter.
__device__ __forceinline__ float jacobi_inv(float M, float floor_, const float* scale, int64_t i) {
    if (!(M > 0.0f)) return 0.0f;
    const float s = scale ? scale[i] : 1.0f;
    return s / fmaxf(M, floor_);
}

// ---- cache element storage -------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
    // The float32 value is rounded again to binary16 (two roundings, like
    // the other storage types); the empty asm keeps the compiler from
    // folding a preceding float64 -> float32 conversion into one
    // float64 -> binary16 rounding.
    asm volatile("" : "+v"(f));
    _Float16 h = (_Float16)f;   // round-to-nearest-even conversion
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// Encode / decode one cached value for storage type DT.
template <int DT> struct Store;
template <> struct Store<LM_CACHE_F32> {
    using word = uint32_t;
    __device__ static word enc(float v) { return __float_as_uint(v); }
    __device__ static float dec(word w) { return __uint_as_float(w); }
    __device__ static word enc_T(float T, bool head, bool clamp) {
        return __float_as_uint(T) | (head ? kHeadBit32 : 0u) | (clamp ? kClampBit32 : 0u);
    }
    __device__ static float dec_T(word w) { return __uint_as_float(w & 0x3FFFFFFFu); }
    __device__ static bool head(word w) { return (w & kHeadBit32) != 0; }
    __device__ static bool clamp(word w) { return (w & kClampBit32) != 0; }
};
template <> struct Store<LM_CACHE_BF16> {
    using word = uint16_t;
    __device__ static word enc(float v) { return f32_to_bf16_rne(v); }
    __device__ static float dec(word w) { return bf16_to_f32(w); }
    __device__ static word enc_T(float T, bool head, bool clamp) {
        return (word)(f32_to_bf16_rne(T) | (head ? kHeadBit16 : 0) | (clamp ? kClampBit16 : 0));
    }
    __device__ static float dec_T(word w) { return bf16_to_f32((uint16_t)(w & 0x3FFFu)); }
    __device__ static bool head(word w) { return (w & kHeadBit16) != 0; }
    __device__ static bool clamp(word w) { return (w & kClampBit16) != 0; }
};
template <> struct Store<LM_CACHE_F16> {
    using word = uint16_t;
    __device__ static word enc(float v) { return f32_to_f16_rne(v); }
    __device__ static float dec(word w) { return f16_to_f32(w); }
    __device__ static word enc_T(float T, bool head, bool clamp) {
        return (word)(f32_to_f16_rne(T) | (head ? kHeadBit16 : 0) | (clamp ? kClampBit16 : 0));
    }
    __device__ static float dec_T(word w) { return f16_to_f32((uint16_t)(w & 0x3FFFu)); }
    __device__ static bool head(word w) { return (w & kHeadBit16) != 0; }
    __device__ static bool clamp(word w) { return (w & kClampBit16) != 0; }
};

inline size_t dtype_bytes(int dt) { return dt == LM_CACHE_F32 ? 4 : 2; }

// ---- launchers implemented in the .hip files --------------------------------
// scan.hip
hipError_t exclusive_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, void* tmp,
                                     size_t tmp_bytes, hipStream_t s);   // out has n+1 entries
size_t scan_tmp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                            int64_t n, int begin_bit, int end_bit, void* tmp, size_t tmp_bytes,
                            bool* result_in_alt, hipStream_t s);
hipError_t radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                                int begin_bit, int end_bit, void* tmp, size_t tmp_bytes, bool* result_in_alt,
                                hipStream_t s);
size_t radix_tmp_bytes(int64_t n);
hipError_t view_sum_f64(const CamDev* cams, int V, const double* in, double* out, hipStream_t s);
hipError_t reduce_f64(const double* in, int64_t n, double* out, hipStream_t s);


// Float64 projection record per (Gaussian, view): mx, my, A, B, C, o, log
// threshold, r, g, b, padded to 16 doubles so that a record is one aligned
// 128-byte line (the raster passes gather one record per tile key).
constexpr int kRecStride = 16;
// A tile is left out of a splat's binning when the splat's exponent stays
// below its alpha threshold by this margin at every pixel centre of the tile.
constexpr double kCullMargin = 1e-3;

// Arguments of the raster passes (raster.hip).
struct RasterArgs {
    const CamDev* cams;
    const int32_t* tile_view;
    const int64_t* tile_start;
    const uint32_t* vals;
    const double* rec64;       // [V*N][kRecStride]
    int64_t N;
    int32_t V, TW, TH;
    // count pass
    int32_t layout;            // 1: a build (per-entry counts, (g, v) counts, block layout); 0: render only
    const float* target;       // [V][3][H][W] or nullptr (render only)
    uint32_t* entry_cnt;       // [K]
    double* pixC;              // [3][n_pix]
    int32_t* ncontrib;         // [n_pix]
    uint32_t* pix_stop;        // [n_pix] build: tile-relative key at which the pixel saturated (~0u: never)
    float* resid;              // image layout
    double* fsq_part;          // [n_tiles]
    uint32_t* tile_pairs;      // [n_tiles] padded pair count
    uint32_t* tile_blk;        // [n_tiles][4] padded pair count per pixel block (count: out, fill: in)
    uint32_t* tile_segs;       // [n_tiles]
    uint32_t* tile_real;       // [n_tiles] real pair count
    uint32_t* gv_cnt;          // [N*V] segments per (g, v), index g*V + v
    int64_t n_pix;
    // fill pass
    const int64_t* tile_pair_off;
    const int64_t* tile_seg_off;
    const uint64_t* gv_idx;    // [N*V+1] exclusive scan of (gv_cnt > 0)
    const uint64_t* gv_segoff; // [N*V+1] exclusive scan of gv_cnt
    uint32_t* gv_cursor;       // [n_gv]
    uint32_t* gv_segs;         // [n_seg]
    void* pT;
    void* pD;                  // [3][pair_stride]
    int64_t pair_stride;
    uint8_t* ppix;
    uint32_t* seg_gv;
    float* seg_f;              // [6][seg_stride]
    int64_t seg_stride;
    uint32_t* run_seg;         // [pair_stride / 8] segment of each aligned 8-pair run
    // thinned cache (thin_k = K > 0; tile_pair_off / tile_blk count pieces)
    int32_t thin_k;
    uint32_t* tile_ck;         // count: [n_tiles] checkpoints per tile
    const int64_t* tile_ck_off;// fill: [n_tiles + 1]
    uint32_t* pix_ck;          // fill: [n_pix] first checkpoint of each pixel in its tile's range
    float* ck;                 // fill: float4 [n_ck]: T, S0, S1, S2 in front of every K-th contributor
    uint32_t* piece_seg;       // fill: [n_pieces] segment of each piece
    uint64_t* piece_mask;      // fill: [n_pieces] contributing pixels of the block (lane bits)
    uint64_t* piece_cmask;     // fill: [n_pieces] those with a clamped alpha
};

// Arguments of the product kernels (apply.hip).
struct ApplyArgs {
    CacheView c;
    const float* x;          // [P][N] parameters the cache was built at
    const float* p;          // [P][N] direction (J modes)
    const float* uin;        // image layout (J^T only)
    float* uout;             // image layout (J only)
    float* dyc;              // [n_gv][9] power coefficients of J_y p
    float* gmom;             // [n_seg][9] moments of J^T u per segment
    float* gvsum;            // [n_gv][9] moments per (Gaussian, view)
    double* gvc;             // chain: [11][lin_stride] float64 + [3K][lin_stride] float32 per gv
    float* edge;             // [2 * waves][9] pieces of gv lists that cross waves
    uint32_t* edge_key;      // [waves]
    double* jp_part;         // [n_tiles] ||J p||^2 per tile
    const int32_t* stop;     // optional device flag: skip when non-zero
    const float* M;          // chain: damping diagonal (or null)
    float* out;              // chain: [P][N] result
    double* pg_part;         // chain: per-block p . out partials (or null)
};

// Product arguments of up to kMaxBatch image subsets of one scene (same
// N, SH degree and cache type): one launch per kernel covers them all; the
// tile pass takes the subsets' tiles one after another (tile_off), the
// other kernels take the subset from blockIdx.y.
constexpr int kMaxBatch = 8;
struct ApplyBatch {
    ApplyArgs a[kMaxBatch];
    int64_t tile_off[kMaxBatch + 1];
    int32_t n;
    float scale, lambda, diag_floor;
};
static_assert(sizeof(ApplyBatch) <= 4000, "kernel argument block too large");

// Device-resident PCG scalars of one subset (pcg.hip).
struct PcgState {
    double rz, rr, bb, pg, alpha, beta;
    int32_t stop, iters, status, pad;
    double hist[LM_PCG_MAX_HISTORY];
};

// persist.hip: the iterations of Algorithm 1 for a batch in one cooperative
// launch (per-subset vectors; the products' arguments are B's)
constexpr int kPersistMaxGrid = 2048;
struct PersistSubset {
    float* x;                // the solution (Algorithm 1's x, the direction delta)
    float* r;
    float* z;
    float* p;                // the search direction (also B.a[b].p)
    const float* M;
    const float* scale;      // learned factors of M^-1, or null
    PcgState* st;
};
struct PersistArgs {
    ApplyBatch B;            // products p -> out (= g); stop flags unused
    PersistSubset v[kMaxBatch];
    int64_t n;               // parameters per subset (N * P)
    int32_t n_iters, tol_mode;
    double tol;
    float floor_;
    uint32_t* bar;           // grid barrier counter (zeroed by the launch)
    int32_t* err;            // set when a grid barrier timed out (zeroed by the launch)
    uint32_t* tile_ctr;      // tile counter of each iteration (zeroed by the launch)
    double* part;            // [kMaxBatch][3][grid] workgroup partial sums
};
int persistent_tile_kind(int dtype, bool thin);
// workgroups that fit on the device at once, and the workgroup size
hipError_t persistent_grid(int deg, int tile, int* grid, int* nt);
// zeroes counters[0 .. n_counters) (barrier, error flag, tile counters),
// then launches the cooperative kernel on dev_args
hipError_t launch_pcg_persistent(const PersistArgs* dev_args, uint32_t* counters, int n_counters, int deg, int tile,
                                 int grid, hipStream_t s);

// project_bin.hip
hipError_t launch_project(const CamDev* cams, const float* x, int64_t N, int V, int deg, int TW, int TH,
                          double* rec64, float* recf, int32_t* rad, uint32_t* keycnt, hipStream_t s);
hipError_t launch_record_keys(const float* recf, const uint32_t* keycnt, int64_t N, int V, uint64_t* rkeys,
                              uint32_t* rvals, hipStream_t s);
hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* keycnt, int64_t R, uint32_t* cnt_sorted,
                                hipStream_t s);
// binning in two launches: the tile test's ballots (kept_mask, of
// bin_mask_words(K, R) words for K rectangle keys) and kept keys per block of
// bin_emit_blocks(R), then (after an exclusive scan of the counts into
// kept_off) the kept keys
int64_t bin_emit_blocks(int64_t R);
int64_t bin_mask_words(int64_t K, int64_t R);
hipError_t launch_bin_count(const CamDev* cams, int64_t N, int64_t R, int TW, int TH, const float* recf,
                            const int32_t* rad, const uint32_t* order, const uint64_t* off_sorted,
                            const double* rec64, uint64_t* kept_mask, uint32_t* kept_blk, hipStream_t s);
hipError_t launch_bin_emit(const CamDev* cams, int64_t N, int64_t R, int TW, int TH, const float* recf,
                           const int32_t* rad, const uint32_t* order, const uint64_t* off_sorted,
                           const double* rec64, uint64_t* kept_mask, const uint64_t* kept_off, int64_t n_kept,
                           uint32_t* keys, uint32_t* vals, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* keys, int64_t K, int64_t n_tiles, int64_t* tile_start,
                              hipStream_t s);
// raster.hip
hipError_t launch_raster(bool fill, int dtype, int64_t n_tiles, const RasterArgs& a, hipStream_t s);
hipError_t launch_flag_nonzero(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s);
hipError_t launch_gv_compact(const uint32_t* gv_cnt, const uint64_t* gv_idx, const uint64_t* gv_segoff, int64_t N,
                             int V, uint32_t* gv_rec, uint32_t* gv_seg_off, uint32_t* gv_first, hipStream_t s);
hipError_t launch_seg_pos(const uint32_t* gv_segs, const uint32_t* seg_gv, int64_t n_seg, uint32_t* seg_pos,
                          uint32_t* list_gv, hipStream_t s);
hipError_t launch_gv_sort(const uint32_t* gv_seg_off, int64_t n_gv, uint32_t* gv_segs, hipStream_t s);
// apply.hip (mode 1 = J, 2 = J^T, 3 = fused J^T J)
hipError_t launch_tangent(const ApplyBatch& B, hipStream_t s);
hipError_t launch_apply_tile(int mode, const ApplyBatch& B, hipStream_t s);
hipError_t launch_chain(const ApplyBatch& B, hipStream_t s);
unsigned chain_blocks(int64_t N);
// Per-segment Gram values (43 floats) reduced per (Gaussian, view) into gvgram.
constexpr int kGramValues = 43;
hipError_t launch_gram(const CacheView& c, float* gram, float* gvgram, float* edge, uint32_t* edge_key,
                       hipStream_t s);
// geo: scratch of 11 doubles per (Gaussian, view) record ([11][lin_stride])
hipError_t launch_jacobi_diag(const CacheView& c, const float* gvgram, double* geo, float* M, hipStream_t s);
hipError_t launch_coverage(const CacheView& c, const float* gvgram, float* coverage, hipStream_t s);
// out 0: dense blocks [n][P][P] of the selected Gaussians, or without a
// selection of the n_sel Gaussians from g0 on; out 1: targets and mask [P][N]
hipError_t launch_block_rows(const CacheView& c, const float* gvgram, const int64_t* sel, int64_t n_sel, int out,
                             float lam, float floor_, float* o0, float* o1, hipStream_t s, int64_t g0 = 0);
// t <- mu_j + beta (t - mu_j) on observed entries; scratch: shrink_scratch_doubles(P)
int64_t shrink_scratch_doubles(int P);
hipError_t launch_target_shrink(float* t, const float* mask, int64_t N, int P, float beta, double* scratch,
                                hipStream_t s);
int64_t feature_parts(int64_t N);   // part holds 12 * feature_parts(N) + 6 doubles
hipError_t launch_precond_features(const float* M, const float* coverage, const float* x, int64_t N, int P,
                                   float* feat, double* part, hipStream_t s);
// mlp.hip
constexpr int kMlpParams = 8896;   // W1 [8][64], b1, W2 [64][64], b2, W3 [64][64], b3 (float32)
hipError_t launch_mlp_forward(const float* w, const float* feat, int64_t n, int p_out, float* s_out, float* scale_out,
                              uint32_t* n_fallback, hipStream_t s);
// gpart holds mlp_grad_parts() * kMlpParams floats, lpart 2 * mlp_grad_parts() doubles
hipError_t launch_mlp_grad_step(float* w, float* adam_m, float* adam_v, int step, float lr, const float* feat,
                                const float* target, const float* mask, int64_t n, int p_out, float* grad_out,
                                double* loss_out, float* gpart, double* lpart, hipStream_t s);
int mlp_grad_parts();
hipError_t launch_gv_reduce_moments(const ApplyBatch& B, hipStream_t s);
// thin.hip: the pair passes of a thinned cache (mode as launch_apply_tile)
hipError_t launch_thin_tile(int mode, const ApplyBatch& B, hipStream_t s);
hipError_t launch_thin_gram(const CacheView& c, float* gram, hipStream_t s);
int64_t gv_reduce_waves(int64_t n_seg);
hipError_t launch_linearize(const CacheView& c, const float* x, float* lin, hipStream_t s);
// objective.hip: residual terms of one view (w, e may be null); part[part0 ..
// part0 + objective_blocks(W, H)) receives the workgroups' sums of E.
struct ObjectiveArgs {
    const float* a;          // image, or the residual image - target when add_target
    const float* t;          // target
    float* w;                // residual weights (or null)
    float* e;                // colour-space residual gradient (or null)
    double* part;
    int64_t off;             // first element of the view ([3][H][W] from here)
    int64_t part0;
    int32_t W, H, kind, add_target;
    double lam1, lam2, eps;
    double g[11];            // 1-D window weights (objective_window)
};
int64_t objective_blocks(int W, int H);
void objective_window(double* g);
hipError_t launch_objective(const ObjectiveArgs& a, hipStream_t s);
// out[v] = E of view v from the partials of launch_objective over views 0..V-1
hipError_t launch_objective_view_sums(const CamDev* cams, int V, const double* part, double* out, hipStream_t s);
// pcg.hip
// Block-Jacobi factors: packed lower Cholesky factors of the damped
// per-Gaussian blocks, element t = i (i + 1) / 2 + j (1 / L_ii in the
// diagonal slots) in tiles of 64 Gaussians, L[g / 64][t][g % 64];
// bj == null means Jacobi.
struct BlockPrecond {
    const float* L;
    int64_t N;
    int P;
};
int64_t pcg_partial_count(int64_t n);
hipError_t pcg_init(int64_t n, const float* b, const float* M, float floor_, const float* scale, float* x,
                    hipStream_t s, const BlockPrecond* bj = nullptr);
hipError_t pcg_init_r(int64_t n, const float* b, const float* g, const float* M, float floor_, const float* scale,
                      float* r, float* z, float* p, double* part, PcgState* st, hipStream_t s,
                      const BlockPrecond* bj = nullptr);
hipError_t pcg_alpha(const double* pg_part, int64_t nb, PcgState* st, hipStream_t s);
hipError_t pcg_update(int64_t n, PcgState* st, float* p, const float* g, const float* M, float floor_,
                      const float* scale, float* x, float* r, float* z, double* part, double tol, int tol_mode,
                      hipStream_t s, const BlockPrecond* bj = nullptr);
// apply.hip: block-Jacobi factors of every Gaussian into L (64-Gaussian tiles)
hipError_t launch_bj_factor(const CacheView& c, const float* gvgram, float lam, float floor_, float* L,
                            uint32_t* n_fallback, hipStream_t s);
hipError_t launch_bj_apply(const BlockPrecond& bj, const float* r, float* z, hipStream_t s);
hipError_t launch_combine(int n_b, const float* const* d, const float* const* m, int64_t n, float* out,
                          hipStream_t s);
// a . b in float64 into out (dev); part holds dot_partial_count(n) doubles
int64_t dot_partial_count(int64_t n);
hipError_t launch_dot(const float* a, const float* b, int64_t n, double* part, double* out, hipStream_t s);
// lm_vec_dot_static: this device's static partial-sum array (looked up on
// first use per device) and its capacity in partial sums
hipError_t dot_static_scratch(double** out);
int64_t dot_static_capacity();
// out = x + gamma d (float32, one rounding)
hipError_t launch_axpy(const float* x, const float* d, float gamma, int64_t n, float* out, hipStream_t s);

}  // namespace lm
