/*
 * lm3dgs.h - C ABI of the MI355X (gfx950) hot path of the Levenberg-Marquardt
 * optimiser for 3D Gaussian Splatting ("3DGS-LM", arXiv 2409.12892).
 *
 * The library solves the damped normal equations of one LM iteration,
 *     (J^T J + lambda diag(J^T J)) delta = -J^T F          (paper eq. norm-eq)
 * with matrix-free Jacobi-preconditioned conjugate gradients (Algorithm 1),
 * where J is the Jacobian of the rendered pixel colours with respect to all
 * Gaussian parameters and F the per-pixel, per-channel residuals
 * F = rendered - target (least-squares colour residuals; supplement A.4 notes
 * dr/dc = 1 for L2).  J p and J^T u are evaluated from a per-pixel,
 * per-splat gradient cache filled once per LM iteration (section 3.3,
 * "Cache-driven parallelization").
 *
 * Conventions
 *   - Every call returns an lm_status: 0 = LM_OK, < 0 error, > 0 warning.
 *     lm_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses this boundary.
 *   - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *     pointers are ordinary host memory.  The library never frees caller
 *     memory.  The device memory a cache or workspace holds comes from the
 *     allocator of the context it was built with (lm_ctx_create; hipMalloc
 *     when the context has none) and goes back to that allocator in
 *     lm_cache_destroy().
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Work is enqueued on it and returns asynchronously unless a
 *     call says it synchronises.
 *   - Parameter vectors (x, p, g, b, M, delta) use the per-attribute
 *     structure-of-arrays layout x[P][N] (paper supplement A.3, vector "q"),
 *     float32, with P = 11 + 3 (deg+1)^2 parameters per Gaussian in the order
 *     mean(3), log-scale(3), quaternion w,x,y,z (4), opacity logit (1),
 *     SH coefficients (index 11 + 3k + channel).
 *   - Images and residual vectors are float32 [V][3][H][W] (view-major,
 *     channel, row, column), all views of one subset back to back.
 */
#ifndef LM3DGS_H
#define LM3DGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lm_status;

enum {
    LM_OK = 0,
    LM_ERR_INVALID_ARG = -1,   /* a pointer, size or option is out of range   */
    LM_ERR_HIP = -2,           /* a HIP runtime call failed (message has it)  */
    LM_ERR_CAPACITY = -3,      /* a size exceeds an index range of the layout */
    LM_ERR_NOT_BUILT = -4,     /* the cache handle is empty                   */
    LM_ERR_UNSUPPORTED = -5,   /* option combination not implemented          */
    LM_WARN_BREAKDOWN = 1,     /* PCG stopped early on p^T A p <= 0 / NaN     */
    LM_WARN_FALLBACK_JACOBI = 2 /* a learned or block preconditioner fell back
                                   to the Jacobi scaling for some parameters  */
};

enum { LM_CACHE_F32 = 0, LM_CACHE_BF16 = 1, LM_CACHE_F16 = 2 };

/* PCG stopping rule.  PAPER_SQUARED is Algorithm 1 as printed:
 * stop when ||r||^2 < tol ||b||^2 (tol = 0.01 in the paper).  RELATIVE stops
 * when ||r|| < tol ||b||.  NONE runs exactly n_iters iterations. */
enum { LM_TOL_NONE = 0, LM_TOL_PAPER_SQUARED = 1, LM_TOL_RELATIVE = 2 };

/* Pinhole camera, world -> camera: X_cam = R X + t (R row-major).  Camera
 * axes x right, y down, z forward; pixel u = fx X/Z + cx, v = fy Y/Z + cy,
 * pixel (i, j) has its centre at (i + 0.5, j + 0.5). */
typedef struct lm_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t W, H;
} lm_camera;

/* The Gaussians: x is a device pointer to float32 [P][N] (see above). */
typedef struct lm_scene {
    int64_t N;
    int32_t sh_degree;    /* 0..3 */
    int32_t reserved;
    const float* x;       /* dev */
} lm_scene;

typedef struct lm_ctx lm_ctx;       /* opaque, library-owned (lm_ctx_create) */

typedef struct lm_options {
    int32_t tile_w, tile_h;  /* tile shape in pixels: tile_w a power of two, tile_w*tile_h
                                <= 256 (0 selects 16)                                     */
    int32_t cache_dtype;     /* LM_CACHE_F32 / _BF16 / _F16 storage of the cache      */
    int32_t flags;           /* 0 or LM_BUILD_COMPACT                                  */
    struct lm_cache** scratch; /* LM_BUILD_COMPACT only: NULL, or the address of a handle
                                  that keeps the build-only buffers between compact builds
                                  (created on first use when *scratch is NULL; release it
                                  with lm_cache_destroy)                                 */
    lm_ctx* ctx;             /* context of the call and of the handles it builds; NULL:
                                the process-wide default context                      */
    int32_t thin_window;     /* 0: the full cache (T and dC/dalpha of every pair).  K in
                                1..LM_THIN_WINDOW_MAX: a thinned cache (section 4.4,
                                limitations: gradients kept only for every K-th splat along
                                a ray, the alpha blending redone inside those windows); it
                                keeps per 64-pixel block and splat a mask of the pixels it
                                contributes to, per pixel the blend state in front of its
                                contributors 0, K, 2K, ..., and no per-pair value; the
                                products re-blend every pair in float32.  Needs
                                LM_CACHE_F32 (else LM_ERR_UNSUPPORTED); the pair exports
                                return LM_ERR_UNSUPPORTED                              */
    int32_t reserved;
} lm_options;
#define LM_THIN_WINDOW_MAX 4096

/* lm_options.flags: after a successful lm_build_cache, synchronise the stream
 * and free the buffers only the build uses (projection records, binning keys
 * and sort buffers, per-pixel counts, residual image), keeping what the
 * products, the diagonal, PCG and the per-view residual norms read; for
 * several subsets resident at once.  A later build on the same handle
 * allocates them again.  lm_cache_export of the pair arrays still works;
 * of the records, sorted values, tile ranges, image, contribution counts
 * and residual it returns LM_ERR_INVALID_ARG.
 * With opts->scratch set, the build borrows the build-only buffers held by
 * *scratch and hands them back afterwards instead of freeing them, so that
 * compact builds of several subsets (each cache then holding only what the
 * products read) allocate their transients once.  Builds sharing one
 * scratch handle must be ordered (one stream, or synchronised); *scratch
 * is never a built cache (products on it return LM_ERR_NOT_BUILT). */
#define LM_BUILD_COMPACT 1

typedef struct lm_cache lm_cache;   /* opaque, library-owned */

/* Device memory allocator: alloc(user, bytes, stream) returns a device
 * buffer for work ordered on `stream` (the hipStream_t of the call that
 * needs it) or NULL on failure (the call then fails with LM_ERR_HIP);
 * free(user, ptr, stream) takes it back on the same stream.  A buffer always
 * goes back to the allocator that supplied it. */
typedef struct lm_allocator {
    void* user;
    void* (*alloc)(void* user, size_t bytes, void* stream);
    void (*free)(void* user, void* ptr, void* stream);
} lm_allocator;

/* A library context holds the allocator of every device buffer allocated on
 * its behalf (caches, workspaces, the autotuner's vectors, lm_vec_dot's
 * partial sums), the PCG launch mode (lm_pcg_use_graph) and the profiling
 * records (lm_profile_*).  A cache or workspace handle belongs to the context
 * of the call that last built it (lm_options.ctx), and every later call on
 * it runs in that context.  Contexts are independent: two contexts in one
 * process give the same results.
 *   lm_ctx_create: allocator (host, copied) may be NULL for hipMalloc /
 *     hipFree; *out receives the context.
 *   lm_ctx_destroy: fails with LM_ERR_INVALID_ARG while handles of the
 *     context are alive (destroy them first) or for the default context;
 *     NULL is a no-op. */
lm_status lm_ctx_create(const lm_allocator* allocator, lm_ctx** out);
lm_status lm_ctx_destroy(lm_ctx* ctx);

/* Installs a (copy of the) allocator in the process-wide default context
 * (lm_options.ctx == NULL); NULL restores hipMalloc / hipFree.  Buffers
 * already allocated keep their allocator. */
lm_status lm_set_allocator(const lm_allocator* allocator);

typedef struct lm_cache_info {
    int64_t N, n_keys, n_pairs, n_segments, n_gv, n_pixels, n_tiles;
                             /* n_keys: (splat, tile) keys kept by the binning;
                                a tile of a splat's rectangle where it stays
                                below its alpha threshold (alpha < 1/255, the
                                alpha-blending equation's skip) is not a key */
    int64_t n_pair_slots;    /* pair storage incl. the zero padding of each piece (a
                                splat's pairs in one 64-pixel block of a tile) to a
                                multiple of 8 pairs                             */
    int64_t cache_bytes;     /* pair + segment arrays read by the products   */
    int64_t device_bytes;    /* all device memory held by the cache          */
    int32_t V, P, tile_w, tile_h, cache_dtype, sh_degree;
    int32_t thin_window;     /* lm_options.thin_window of the build (0: full cache)  */
    int32_t reserved;
    int64_t n_pieces;        /* thinned cache: (splat, 64-pixel block) pieces         */
    int64_t n_checkpoints;   /* thinned cache: stored blend states                    */
} lm_cache_info;

#define LM_PCG_MAX_HISTORY 257
typedef struct lm_pcg_stats {
    int32_t iters;           /* completed loop iterations                        */
    int32_t status;          /* LM_OK or LM_WARN_BREAKDOWN                       */
    double b_sqnorm;         /* ||b||^2                                          */
    double history[LM_PCG_MAX_HISTORY];  /* ||r_i||^2 / ||b||^2, i = 0..iters      */
} lm_pcg_stats;

/* Message for the last error on this thread ("" if none). */
const char* lm_last_error(void);

/* Build the per-pixel, per-splat gradient cache of one image subset
 * (Algorithm 1, buildCache; section 3.3 "Mapping of PCG to CUDA kernels").
 * Projects every Gaussian into the V views, bins and depth-sorts the splats
 * per tile, alpha-blends every pixel (eq. alpha-blending), writes the cache
 * and forms b = -J^T F.
 *   scene, cams (host, V entries), target (dev float32 [V][3][H][W]).
 *   *inout: NULL to create a new cache, or an existing cache whose device
 *           memory is reused (grown when needed).
 *   b (dev float32 [P][N], may be NULL), F_sqnorm (dev double, may be NULL).
 * Synchronises the stream twice (to size the key and pair arrays). */
lm_status lm_build_cache(const lm_scene* scene, const lm_camera* cams, int32_t V,
                         const float* target, const lm_options* opts, void* stream,
                         lm_cache** inout, float* b, double* F_sqnorm);

lm_status lm_cache_destroy(lm_cache* cache);
lm_status lm_cache_get_info(const lm_cache* cache, lm_cache_info* info);

/* Device memory held by each buffer of the cache, for sizing a set of
 * resident caches: entry i gets the buffer's name (NUL-terminated) and the
 * bytes it holds (0 for a buffer never allocated or released).  out (host,
 * capacity entries, may be NULL when capacity is 0) receives the first
 * min(capacity, *n) entries; *n (host) is set to the number of buffers. */
typedef struct lm_buffer_bytes {
    char name[24];
    uint64_t bytes;
} lm_buffer_bytes;
lm_status lm_cache_memory(const lm_cache* cache, lm_buffer_bytes* out, int32_t capacity, int32_t* n);

/* Synchronises the stream and frees what the products and lm_pcg_solve do
 * not read: the per-(Gaussian, view) Gram values behind the diagonal, the
 * learned-preconditioner inputs and the block-Jacobi factors, with their
 * scratch.  A later call that needs them computes them again.  For caches
 * held resident together (with LM_BUILD_COMPACT).  On a compact cache the
 * per-(splat, tile) Gram values, reduced per (Gaussian, view) right after
 * they are formed, are never kept. */
lm_status lm_cache_trim(lm_cache* cache, void* stream);

/* M = diag(J^T J) (paper eq. diag-jtj, kernel diagJTJ), dev float32 [P][N].
 * With residual weights set on the cache (lm_set_residual_weights,
 * lm_cache_objective) every product below uses J^T W J in place of J^T J
 * (supplement A.4, eq. apply-jtj-simplified-vec-vec): this diagonal, the
 * J^T J half of lm_apply_JtJ and lm_pcg_solve, and the squared norms
 * (sum w (J p)^2).  lm_apply_J and lm_apply_JT stay the plain colour
 * Jacobian products. */
lm_status lm_jacobi_diag(const lm_cache* cache, float* M, void* stream);

/* g = J^T J p + lambda M p (Algorithm 1, the applyJ / applyJT pair plus the
 * damping term).  M may be NULL (then lambda is ignored).  If Jp_sqnorm is
 * not NULL, ||J p||^2 (double, dev) is written too.  p, g dev [P][N]. */
lm_status lm_apply_JtJ(const lm_cache* cache, const float* p, float lambda, const float* M,
                       float* g, double* Jp_sqnorm, void* stream);

/* u = J p (eq. apply-j), u dev float32 [V][3][H][W]. */
lm_status lm_apply_J(const lm_cache* cache, const float* p, float* u, void* stream);

/* ||J p||^2 (float64, dev, one value): the J product alone, with the
 * squared norm of each tile's u summed in a fixed order (the denominator of
 * the trust-region ratio, eq. tr-update, needs no J^T half). */
lm_status lm_jp_sqnorm(const lm_cache* cache, const float* p, double* out, void* stream);

/* g = J^T u (eq. apply-jt), u dev float32 [V][3][H][W], g dev [P][N]. */
lm_status lm_apply_JT(const lm_cache* cache, const float* u, float* g, void* stream);

/* ---- the paper's objective (section 3.1 eq. sgd-loss, eq. gn-loss;
 * supplement A.4) ----
 * Per pixel and colour channel, residuals r1 = sqrt(lambda1 |c - C|) and
 * r2 = sqrt(lambda2 (1 - SSIM(c, C))); E = sum r1^2 + r2^2.  SSIM per
 * channel: 11 x 11 Gaussian window of standard deviation 1.5 (weights sum to
 * 1, pixels outside the image are 0), C1 = 0.01^2, C2 = 0.03^2; its
 * derivative goes to the window's centre pixel only (section 3.3).  The
 * Gauss-Newton system needs two images: the colour-space gradient
 * e = sum_t r_t dr_t/dc (b = -J^T e) and the residual weight
 * w = sum_t (dr_t/dc)^2 = sum_t f_t'^2 / (4 max(f_t, eps)), f_t = r_t^2.
 * LM_OBJ_L2 is the plain least-squares objective r = c - C (e = r, w = 1). */
enum { LM_OBJ_L2 = 0, LM_OBJ_L1_SSIM = 1 };
typedef struct lm_objective {
    int32_t kind;            /* LM_OBJ_L2 or LM_OBJ_L1_SSIM                      */
    float lambda1, lambda2;  /* 0.8 and 0.2 in the paper                         */
    float eps;               /* floor of f_t in the weight's denominator, > 0    */
} lm_objective;

/* Terms of the objective for images already in device memory: image and
 * target dev float32 [V][3][H][W] (view sizes from cams).  w and e (same
 * layout) may be NULL; E (dev double, one value) is written.  Enqueued on
 * the stream; *workspace as for lm_residual_sqnorm (NULL or a reusable
 * handle; the call keeps its partial sums there).  Errors: NULL image,
 * target, E or workspace, V < 1, an unknown kind, eps <= 0. */
lm_status lm_objective_terms(const float* image, const float* target, const lm_camera* cams, int32_t V,
                             const lm_objective* obj, float* w, float* e, double* E, void* stream,
                             lm_cache** workspace);

/* Set the cache's residual weights, dev float32 [V][3][H][W] of the cache's
 * views (copied; the caller keeps ownership of w).  w == NULL returns to
 * plain least squares (unit weights). */
lm_status lm_set_residual_weights(lm_cache* cache, const float* w, void* stream);

/* The objective at the point the cache was built at (its rendered image is
 * the stored residual plus target, the same target as the build): sets the
 * cache's residual weights (NULL weights for LM_OBJ_L2), writes
 * b = -J^T e (dev float32 [P][N], may be NULL) and E (dev double, may be
 * NULL).  With LM_OBJ_L2, b and E equal the build's b and ||F||^2. */
lm_status lm_cache_objective(lm_cache* cache, const float* target, const lm_objective* obj, float* b,
                             double* E, void* stream);

/* The objective of a forward render (line search of the LM loop, eq.
 * line-search): render the views at the scene's x and evaluate E against
 * target (no cache fill).  *workspace as for lm_residual_sqnorm. */
lm_status lm_objective_value(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                             const lm_options* opts, const lm_objective* obj, void* stream,
                             lm_cache** workspace, double* E);

/* Algorithm 1 for n_b image subsets (section 3.3 "Image Subsampling
 * Scheme": each subset solves its own normal equations).  All arrays are
 * host arrays of n_b device pointers; precond_scale may be NULL (plain
 * Jacobi) or hold per-subset NULL / dev float32 [P][N] factors multiplying
 * M^-1.  diag_floor: 0 runs Algorithm 1 exactly; > 0 replaces every
 * positive diagonal entry below it by the floor in both the damping term
 * and the Jacobi preconditioner (a minimum LM diagonal, as in CERES, whose
 * LM variant the paper follows); unobserved parameters (M = 0) keep a zero
 * update either way.  Dots, alpha and beta are float64 and stay on the
 * device; the stopping test runs on the device.  stats (host, n_b entries)
 * is filled after one synchronisation at the end.
 * Batching: the subsets (at most 8 per call; same N, SH degree and cache
 * type) share every product launch - the tile pass takes all subsets'
 * tiles in one grid - and, with graph replay on (lm_pcg_use_graph), one
 * iteration is captured once and replayed n_iters times. */
lm_status lm_pcg_solve(lm_cache* const* caches, int32_t n_b, const float* const* b,
                       const float* const* M, float lambda, float diag_floor, int32_t n_iters,
                       double tol, int32_t tol_mode, const float* const* precond_scale,
                       float* const* delta, lm_pcg_stats* stats, void* stream);

/* Block-Jacobi preconditioner (a stronger preconditioner than the paper's
 * Jacobi choice of section 3.3): per Gaussian the damped block
 * A_k = J_k^T J_k + lambda diag(max(d, diag_floor)) of eq. norm-eq
 * restricted to the Gaussian's own P parameters (d = diag(J_k^T J_k); a
 * parameter with d = 0 keeps a unit diagonal and no coupling), inverted
 * exactly through a Cholesky factor, in place of M^-1 in Algorithm 1.  The
 * factors (P (P + 1) / 2 floats per Gaussian) are computed on first use for
 * (lambda, diag_floor) and kept in the cache until the next build or
 * residual-weight change; with residual weights the blocks are those of
 * J^T W J.  Same arguments and behaviour as lm_pcg_solve otherwise. */
lm_status lm_pcg_solve_block(lm_cache* const* caches, int32_t n_b, const float* const* b,
                             const float* const* M, float lambda, float diag_floor, int32_t n_iters,
                             double tol, int32_t tol_mode, float* const* delta, lm_pcg_stats* stats,
                             void* stream);

/* z = A^-1 r with the block-Jacobi factors for (lambda, diag_floor) (r, z
 * dev float32 [P][N]).  n_fallback (host, may be NULL): when given, the
 * factors are recomputed and it receives the number of Gaussians whose
 * damped block did not factor (those use their damped diagonal, the Jacobi
 * scaling); the call then synchronises the stream and returns
 * LM_WARN_FALLBACK_JACOBI when the number is not 0. */
lm_status lm_block_precond_apply(lm_cache* cache, float lambda, float diag_floor, const float* r, float* z,
                                 int32_t* n_fallback, void* stream);

/* Tile shape for one image subset, measured: for each candidate shape
 * (16x16, 32x8, 8x32, 16x8, 8x16, 8x8) the cache is built twice (the
 * first build absorbs buffer growth), the second build and two J^T J
 * products (along b) are timed; the shape with the smallest
 * build_ms + n_products * apply_ms is returned in tile_w/tile_h.  scores
 * (host, may be NULL) receives up to max_scores per-candidate timings and
 * n_scores their count.  opts (may be NULL) gives the context, whose
 * allocator supplies the candidates' caches and two parameter vectors
 * (freed before returning), and the cache type; its tile fields are
 * ignored.  Synchronises the stream. */
typedef struct lm_tile_score {
    int32_t tile_w, tile_h;
    float build_ms, apply_ms;
} lm_tile_score;
lm_status lm_autotune_tile(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                           const lm_options* opts, int32_t n_products, void* stream, int32_t* tile_w,
                           int32_t* tile_h, lm_tile_score* scores, int32_t max_scores, int32_t* n_scores);

/* Launch mode of the PCG iterations of a context (NULL: the default
 * context): 0 launches every kernel of every iteration from the host; 1
 * captures one iteration into a graph (on a library-owned stream) and
 * replays it on the caller's stream; 2 (default) uses the graph when a call
 * solves more than one subset; 3 runs all iterations of all subsets of a
 * call in one persistent cooperative kernel (one workgroup per resident
 * slot, grid-wide barriers between the phases of an iteration, the float64
 * scalars formed identically by every workgroup), its launch captured into
 * a graph once per context and kernel variant and replayed (issued directly
 * where the runtime cannot capture a cooperative launch); the call
 * synchronises the stream, and a barrier that does not complete within 10 s
 * ends the kernel and the call returns LM_ERR_HIP.  lm_pcg_solve_block
 * uses mode 2 when 3 is set.  Results agree between modes to float32
 * rounding (modes 0-2 are bit-identical; mode 3 sums the p.g, r.z and r.r
 * partials over its own grid). */
lm_status lm_pcg_use_graph(lm_ctx* ctx, int32_t mode);

/* Vector steps of the LM outer loop (section 3.2), so that no method
 * arithmetic runs outside the library.
 * lm_vec_dot: *out (dev double) = a^T b in float64 for float32 dev vectors
 *   a, b of n elements (NULL allowed when n = 0; then *out = 0); the trust-region ratio's model decrease (eq.
 *   tr-update) is 2 gamma delta^T b - gamma^2 ||J delta||^2 with b = -J^T F.
 *   Partial sums go to device memory of the context (NULL: default),
 *   allocated through its allocator on first use and kept until
 *   lm_ctx_destroy.  Fixed summation order (deterministic).
 * lm_vec_axpy: out = x + gamma d element-wise in float32 (one rounding per
 *   element), the parameter update x_{k+1} = x_k + gamma delta of section
 *   3.2; out may alias x.  Allocates nothing. */
lm_status lm_vec_dot(lm_ctx* ctx, const float* a, const float* b, int64_t n, double* out, void* stream);
lm_status lm_vec_axpy(const float* x, const float* d, float gamma, int64_t n, float* out, void* stream);

/* For callers that cannot allocate device memory (code under stream or
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * float64 dot product as lm_vec_dot, bit-identical to it, with its partial
 * sums in a static device array of the library instead of context memory.
 *   a, b: float32 dev vectors of n elements; out: one dev double.
 *   n <= LM_VEC_DOT_STATIC_MAX_N (2^40), else LM_ERR_CAPACITY.  The array
 *   holds the 2048 per-block partial sums of the fixed vector grid (16 KiB);
 *   every GPU the library runs on holds its own copy until the process ends.
 *   Every element the call reads is written by the same call first, so
 *   nothing needs clearing between calls.
 *   Allocates nothing (no hipMalloc, no allocator call).  All calls on one
 *   GPU share that GPU's array: calls that overlap on one GPU (several
 *   streams or threads without ordering) race and give wrong results. */
#define LM_VEC_DOT_STATIC_MAX_N ((int64_t)1 << 40)
lm_status lm_vec_dot_static(const float* a, const float* b, int64_t n, double* out, void* stream);

/* Weighted mean of subset directions (paper eq. combine-pcg):
 * out = sum_i M_i delta_i / sum_k M_k element-wise; 0 where sum_k M_k = 0.
 * delta, M: host arrays of n_b dev float32 pointers of n elements each. */
lm_status lm_combine_subsets(int32_t n_b, const float* const* delta, const float* const* M,
                             int64_t n, float* out, void* stream);

/* ---- Learned diagonal preconditioner --------------------------------------
 * An extension of the Jacobi preconditioner of Algorithm 1 (section 3.3):
 * a perceptron predicts, per parameter, a log-scale s of the Jacobi inverse,
 * M^-1 = exp(s) / diag(J^T J), passed to lm_pcg_solve as precond_scale.
 * Training data come from the per-Gaussian blocks of J^T J, which the paper
 * does not use; they are built from the same per-(Gaussian, view) Gram
 * values as the Jacobi diagonal (its eq. diag-jtj computes their diagonal).
 * Calls on one cache must be ordered on one stream (they share its Gram
 * buffers, computed once per build). */

/* Number of (pixel, splat) pairs of each Gaussian over all views of the
 * cache, dev float32 [N] (an exact count up to 2^24 per Gaussian). */
lm_status lm_pair_coverage(const lm_cache* cache, float* coverage, void* stream);

/* Dense blocks B_k = J_k^T J_k (P x P, over the P parameters of Gaussian k)
 * of the n Gaussians listed in gaussians (dev int64 [n], each in [0, N);
 * not checked on the device), written to blocks (dev float32 [n][P][P],
 * row-major, symmetric up to rounding). */
lm_status lm_block_jacobi(const lm_cache* cache, const int64_t* gaussians, int64_t n, float* blocks,
                          void* stream);

/* Training targets of the learned preconditioner, dev float32 [P][N] each.
 * For parameter j of Gaussian k with d = (B_k)_jj > 0 and D = max(d,
 * diag_floor), row j of B_k summed over the views in float64 (from the
 * float32 per-(Gaussian, view) Gram values) and the target computed in
 * float64: r = log(D / (sum_i |(B_k)_ji| + lambda D)), the diagonal
 * scaling that bounds the Gershgorin discs of the damped block
 * B_k + lambda diag(D), relative to Jacobi; then t = mu_j + shrink
 * (r - mu_j) with mu_j the mean of r over the observed Gaussians of
 * parameter j (shrink in [0, 1]; 1 keeps r);
 * mask = 1.  Where d = 0: t = 0, mask = 0.  The means are summed in a fixed
 * order (deterministic). */
lm_status lm_precond_targets(const lm_cache* cache, float lambda, float diag_floor, float shrink, float* t,
                             float* mask, void* stream);

/* Eight features per Gaussian, dev float32 [8][N], from the parameters x
 * (dev [P][N]) and the Jacobi diagonal M (dev [P][N], from lm_jacobi_diag):
 * 0-4: log of the mean of M over the mean (3), log-scale (3), quaternion
 * (4), opacity (1) and SH (P - 11) parameters; 5: log(1 + pair count);
 * each centred on its mean over the observed Gaussians (sum of M > 0) where
 * it is finite, else 0; 6: sigmoid of the opacity logit; 7: the mean
 * log-scale.  Unobserved Gaussians get eight zeros. */
lm_status lm_precond_features(const lm_cache* cache, const float* x, const float* M, float* feat, void* stream);

/* Weights: dev float32 [LM_MLP_PARAMS]: W1 [8][64] (input-major), b1 [64],
 * W2 [64][64], b2 [64], W3 [64][64] (columns >= p_out unused), b3 [64].
 * The products run on bfloat16 copies of the weights and activations with
 * float32 accumulation. */
#define LM_MLP_FEATURES 8
#define LM_MLP_HIDDEN 64
#define LM_MLP_MAX_OUT 64
#define LM_MLP_PARAMS 8896

/* s = W3^T gelu(W2^T gelu(W1^T f + b1) + b2) + b3 for n samples (columns
 * of feat, dev [8][n]); 1 <= p_out <= 64.  s (dev [p_out][n]) and scale =
 * exp(clamp(s, -4, 4)) (dev [p_out][n]) may each be NULL.  A non-finite s
 * gives scale 1 (the Jacobi preconditioner) and is counted in n_fallback
 * (dev uint32, may be NULL; set to the count of this call).  With n_fallback
 * given the call synchronises the stream and returns LM_WARN_FALLBACK_JACOBI
 * when the count is not 0. */
lm_status lm_mlp_forward(const float* w, const float* feat, int64_t n, int32_t p_out, float* s, float* scale,
                         uint32_t* n_fallback, void* stream);

/* Device workspace (bytes) lm_mlp_train_step needs, for any n. */
size_t lm_mlp_workspace_bytes(void);

/* One training step on the masked mean squared error
 * L = sum mask (s - target)^2 / sum mask (target, mask dev [p_out][n]):
 * grad (dev float32 [LM_MLP_PARAMS], may be NULL) and loss (dev double, may
 * be NULL) are taken at the weights on entry; then, if lr > 0, one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction with the 1-based
 * step) updates w, adam_m and adam_v (dev [LM_MLP_PARAMS]; zero them before
 * step 1).  The gradient is summed in a fixed order (deterministic).
 * workspace: dev, at least lm_mlp_workspace_bytes(). */
lm_status lm_mlp_train_step(float* w, float* adam_m, float* adam_v, int32_t step, float lr, const float* feat,
                            const float* target, const float* mask, int64_t n, int32_t p_out, float* grad,
                            double* loss, void* workspace, size_t workspace_bytes, void* stream);

/* Forward render only (eq. alpha-blending), image dev float32 [V][3][H][W]. */
lm_status lm_render(const lm_scene* scene, const lm_camera* cams, int32_t V,
                    const lm_options* opts, float* image, void* stream);

/* ||F(x)||^2 = ||render(x) - target||^2 summed over the given views, float64
 * on the device (forward pass only: projection, binning, depth sort and
 * alpha-blending; no cache fill).  Serves the line search (eq. line-search)
 * and the trust-region ratio (eq. tr-update) of the LM outer loop.
 * *workspace: NULL or a handle whose device memory is reused; after the call
 * it holds no usable cache (products on it return LM_ERR_NOT_BUILT). */
lm_status lm_residual_sqnorm(const lm_scene* scene, const lm_camera* cams, int32_t V,
                             const float* target, const lm_options* opts, void* stream,
                             lm_cache** workspace, double* F_sqnorm);

/* Per-view ||F||^2 of a built cache (the residual at the x it was built at,
 * split by view; their sum is the F_sqnorm of lm_build_cache).  Used by
 * the line search of section 3.2 (eq. line-search), which compares errors on
 * a subset of the views.  per_view: dev double [V], written in view order. */
lm_status lm_cache_view_sqnorm(const lm_cache* cache, double* per_view, void* stream);

/* Copy an internal array of a built cache to host memory (inspection and
 * tests).  Synchronises the stream.  `what` selects the array; `bytes` must
 * equal the array's size (lm_cache_export_size()). */
enum {
    LM_EXPORT_RECORDS_F32 = 0,   /* float [V][N][4]: mean x, mean y, depth, radius (as float) */
    LM_EXPORT_SORTED_VALUES = 1, /* uint32 [n_keys]: Gaussian id, tile-major depth order       */
    LM_EXPORT_TILE_RANGES = 2,   /* int64 [n_tiles+1]: start of each tile's list              */
    LM_EXPORT_IMAGE = 3,         /* float [V][3][H][W]: rendered colour                       */
    LM_EXPORT_NCONTRIB = 4,      /* int32 [V][H][W]: contributing splats per pixel            */
    LM_EXPORT_PAIR_T = 5,        /* float [n_pairs]: cached transmittance (flags removed)     */
    LM_EXPORT_PAIR_D = 6,        /* float [3][n_pairs]: cached dC/dalpha                      */
    LM_EXPORT_PAIR_PIX = 7,      /* int32 [n_pairs]: global pixel index v*H*W + y*W + x       */
    LM_EXPORT_PAIR_GAUSS = 8,    /* int32 [n_pairs]: Gaussian id of the pair's splat          */
    LM_EXPORT_RESIDUAL = 9,      /* float [V][3][H][W]: F = rendered - target                 */
    LM_EXPORT_PAIR_FLAGS = 10,   /* int32 [n_pairs]: bit0 first pair of a piece (a splat's
                                    pairs in one pixel block of a tile), bit1 alpha clamped */
    LM_EXPORT_TILE_SEGMENTS = 11 /* int64 [n_tiles+1]: first segment (a splat with pairs in
                                    the tile) of each tile                               */
};
int64_t lm_cache_export_size(const lm_cache* cache, int32_t what);
lm_status lm_cache_export(const lm_cache* cache, int32_t what, void* host_dst, int64_t bytes,
                          void* stream);

/* Opt-in timing of the library's own kernels with HIP events recorded on
 * the stream each kernel is launched on, per context (NULL: the default
 * context; a call records into the context it runs in).
 * lm_profile_enable(ctx, 1) starts recording (one start/stop event pair
 * around every kernel group the library launches), lm_profile_enable(ctx, 0)
 * stops.  lm_profile_read() synchronises on the context's recorded events,
 * returns per-group totals (at most max_entries, sorted by name) and clears
 * the record.  Not thread-safe: meant for a single driver thread. */
typedef struct lm_profile_entry {
    char name[40];
    int32_t launches;
    int32_t reserved;
    double total_ms;
} lm_profile_entry;
lm_status lm_profile_enable(lm_ctx* ctx, int32_t on);
int32_t lm_profile_read(lm_ctx* ctx, lm_profile_entry* out, int32_t max_entries);

#ifdef __cplusplus
}
#endif

#endif /* LM3DGS_H */
