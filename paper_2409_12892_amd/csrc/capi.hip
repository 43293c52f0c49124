// Host side of the C ABI declared in include/lm3dgs.h: cache construction
// and the orchestration of the kernels on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lm_internal.h"

namespace lm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace prof {
// Event pairs recorded around kernel groups while profiling is enabled.
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
struct State {
    bool enabled = false;
    bool capturing = false;   // no event records while a stream is captured
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    hipEvent_t take() {
        if (used < pool.size()) return pool[used++];
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
        ++used;
        return e;
    }
};
}  // namespace prof
}  // namespace lm

// A library context: the allocator of the device memory allocated on its
// behalf, the launch mode of PCG and the profiling records.  Caches belong
// to the context they were built with.
struct lm_ctx {
    lm_allocator al{};
    int pcg_graph = 2;       // 0 eager, 1 graph replay, 2 graph replay for batches, 3 persistent kernel
    // persistent-kernel PCG: device arguments, counters and partials (grown
    // on demand, kept until lm_ctx_destroy) and the captured launch
    void* persist_dev = nullptr;      // PersistArgs, then counters, then partials
    size_t persist_cap = 0;
    lm_allocator persist_al{};
    hipStream_t persist_stream = nullptr;
    hipGraphExec_t persist_exec = nullptr;
    int persist_key[3] = {-1, -1, -1}; // (SH degree, tile variant, grid) of persist_exec
    int persist_graph = -1;           // -1 untried, 0 capture unsupported, 1 captured launches
    lm::prof::State prof;
    int64_t n_caches = 0;    // live caches (and workspaces) bound to the context
    // partial sums of lm_vec_dot (grown on demand, kept until lm_ctx_destroy)
    void* part = nullptr;
    size_t part_cap = 0;
    lm_allocator part_al{};
    hipStream_t part_stream = nullptr;
};

namespace lm {

// The process-wide default context (lm_options.ctx == NULL), and the
// context and stream of the entry point running on this thread: device
// memory is allocated through the context's allocator, stream-ordered on
// the entry point's stream.
static lm_ctx g_default_ctx;
static thread_local lm_ctx* g_ctx = &g_default_ctx;
static thread_local hipStream_t g_alloc_stream = nullptr;
struct StreamScope {
    hipStream_t prev;
    lm_ctx* prevc;
    explicit StreamScope(hipStream_t s, lm_ctx* c = nullptr) : prev(g_alloc_stream), prevc(g_ctx) {
        g_alloc_stream = s;
        if (c) g_ctx = c;
    }
    ~StreamScope() {
        g_alloc_stream = prev;
        g_ctx = prevc;
    }
};

namespace prof {
struct Scope {
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    State& st;
    Scope(const char* n, hipStream_t stream) : name(n), s(stream), st(g_ctx->prof) {
        if (st.enabled && !st.capturing) {
            a = st.take();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Scope() {
        if (st.enabled && !st.capturing && a) {
            hipEvent_t b = st.take();
            if (b) {
                (void)hipEventRecord(b, s);
                st.recs.push_back({name, a, b});
            }
        }
    }
};
}  // namespace prof

#define LM_PROF(name, stream) ::lm::prof::Scope lm_prof_scope_##__LINE__(name, stream)

namespace {

// Device buffer that only grows; reused across rebuilds of one cache.  It
// is returned through the allocator that supplied it, on the stream it was
// allocated on.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    lm_allocator al{};
    hipStream_t st = nullptr;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap && p) return hipSuccess;
        release();
        const size_t want = bytes + bytes / 16 + 256;
        const lm_allocator g = lm::g_ctx->al;
        const hipStream_t s = lm::g_alloc_stream;
        if (g.alloc) {
            p = g.alloc(g.user, want, (void*)s);
            if (!p) return hipErrorOutOfMemory;
        } else {
            hipError_t e = hipMalloc(&p, want);
            if (e != hipSuccess) {
                p = nullptr;
                return e;
            }
        }
        al = g;
        st = s;
        cap = want;
        return hipSuccess;
    }
    void release() {
        if (p) {
            if (al.alloc) al.free(al.user, p, (void*)st);
            else (void)hipFree(p);
        }
        p = nullptr;
        cap = 0;
    }
    template <class T> T* as() const { return (T*)p; }
    void swap(DevBuf& o) {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
        std::swap(al, o.al);
        std::swap(st, o.st);
    }
};

inline int64_t round_up(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

}  // namespace
}  // namespace lm

using lm::DevBuf;

// Every device buffer of a cache (one list for declaration, size report and
// release).
#define LM_CACHE_BUFFERS(X) \
    X(cams) X(tile_view) X(x) X(rec64) X(recf) X(rad) \
    X(keycnt) X(keyoff) X(keys) X(vals) X(keys_alt) X(vals_alt) \
    X(sort_tmp) X(scan_tmp) X(rkeys) X(rvals) X(rkeys_alt) X(rvals_alt) \
    X(cnt_sorted) X(kept_blk) X(kept_off) X(kept_mask) X(tile_start) X(entry_cnt) \
    X(pixC) X(ncontrib) X(pix_stop) X(resid) X(fsq_part) X(tile_pairs) X(tile_segs) \
    X(tile_pair_off) X(tile_seg_off) X(tile_real) X(tile_real_off) X(run_seg) X(gv_cnt) \
    X(gv_flag) X(gv_idx) X(gv_segoff) X(gv_rec) X(gv_seg_off) X(gv_first) \
    X(gv_cursor) X(gv_segs) X(seg_pos) X(list_gv) X(pT) X(pD) \
    X(ppix) X(seg_gv) X(tile_blk) X(seg_f) X(dyc) X(gmom) \
    X(jp_part) X(gram) X(pg_part) X(scalar) X(lin) X(gvsum) \
    X(gvchain) X(edge_m) X(ekey_m) X(gvgram) X(edge_g) X(ekey_g) \
    X(coverage) X(feat_red) X(tgt_red) X(wres) X(obj_e) X(obj_part) \
    X(bj_L) X(bj_count) X(tile_ck) X(tile_ck_off) X(pix_ck) X(ck) \
    X(piece_seg) X(piece_mask) X(piece_cmask) X(pcg_r) X(pcg_z) X(pcg_p) \
    X(pcg_g) X(pcg_part) X(pcg_state)

struct lm_cache {
    lm_ctx* ctx = nullptr;       // the context of its last build (NULL before)
    int64_t N = 0;
    int P = 0, deg = 0, V = 0, TW = 16, TH = 16, dtype = LM_CACHE_F32;
    int64_t n_tiles = 0, n_pix = 0, n_keys = 0, n_pairs = 0, n_slots = 0, n_seg = 0, n_gv = 0;
    int64_t pair_stride = 8, seg_stride = 8, lin_stride = 8;
    int thin_k = 0;                  // > 0: thinned cache (checkpoint every thin_k contributors)
    int64_t n_pieces = 0, n_ck = 0;  // thinned cache: pieces and checkpoints
    bool vals_in_alt = false;
    bool built = false;
    std::vector<lm::CamDev> cams_h;
    std::vector<int> viewW, viewH;
#define LM_DECLARE_BUF(n) DevBuf n;
    LM_CACHE_BUFFERS(LM_DECLARE_BUF)
#undef LM_DECLARE_BUF
    bool weighted = false;       // wres holds residual weights for the products
    bool bj_valid = false;       // bj_L holds the block-Jacobi factors for (bj_lambda, bj_floor)
    float bj_lambda = 0.0f, bj_floor = 0.0f;
    bool gram_valid = false;     // gvgram holds the Gram values of the current build
    bool compact = false;        // the build-only buffers were released (LM_BUILD_COMPACT)

    const uint32_t* sorted_vals() const { return vals_in_alt ? vals_alt.as<uint32_t>() : vals.as<uint32_t>(); }

    lm::CacheView view() const {
        lm::CacheView c{};
        c.N = N; c.P = P; c.deg = deg; c.V = V; c.TW = TW; c.TH = TH; c.dtype = dtype;
        c.tw_shift = 0;
        while ((1 << c.tw_shift) < TW) ++c.tw_shift;
        c.n_tiles = n_tiles; c.n_pix = n_pix; c.n_seg = n_seg; c.n_gv = n_gv;
        c.cams = cams.as<lm::CamDev>();
        c.tile_view = tile_view.as<int32_t>();
        c.tile_pair_off = tile_pair_off.as<int64_t>();
        c.tile_seg_off = tile_seg_off.as<int64_t>();
        c.pT = pT.p; c.pD = pD.p; c.ppix = ppix.as<uint8_t>();
        c.n_pairs = n_slots; c.pair_stride = pair_stride;
        c.run_seg = run_seg.as<uint32_t>();
        c.seg_gv = seg_gv.as<uint32_t>(); c.tile_blk = tile_blk.as<uint32_t>(); c.seg_f = seg_f.as<float>();
        c.seg_stride = seg_stride;
        c.gv_rec = gv_rec.as<uint32_t>(); c.gv_first = gv_first.as<uint32_t>();
        c.gv_seg_off = gv_seg_off.as<uint32_t>(); c.gv_segs = gv_segs.as<uint32_t>();
        c.seg_pos = seg_pos.as<uint32_t>(); c.list_gv = list_gv.as<uint32_t>();
        c.lin = lin.as<float>(); c.lin_stride = lin_stride;
        c.wres = weighted ? wres.as<float>() : nullptr;
        c.thin_k = thin_k;
        c.piece_seg = piece_seg.as<uint32_t>();
        c.piece_mask = piece_mask.as<uint64_t>();
        c.piece_cmask = piece_cmask.as<uint64_t>();
        c.tile_ck_off = tile_ck_off.as<int64_t>();
        c.pix_ck = pix_ck.as<uint32_t>();
        c.ck = ck.as<float4>();
        return c;
    }

    lm::ApplyArgs apply_args() const {
        lm::ApplyArgs a{};
        a.c = view();
        a.x = x.as<float>();
        a.dyc = dyc.as<float>();
        a.gmom = gmom.as<float>();
        a.gvsum = gvsum.as<float>();
        a.gvc = gvchain.as<double>();
        a.edge = edge_m.as<float>();
        a.edge_key = ekey_m.as<uint32_t>();
        a.jp_part = jp_part.as<double>();
        return a;
    }

    size_t device_bytes() const {
        size_t s = 0;
#define LM_ADD_BUF(n) s += n.cap;
        LM_CACHE_BUFFERS(LM_ADD_BUF)
#undef LM_ADD_BUF
        return s;
    }
    // name and bytes held of each buffer, in declaration order
    template <class F>
    void each_buffer(F&& f) const {
#define LM_EACH_BUF(n) f(#n, n.cap);
        LM_CACHE_BUFFERS(LM_EACH_BUF)
#undef LM_EACH_BUF
    }

    // buffers read only while building (see LM_BUILD_COMPACT)
    static constexpr int kBuildBufs = 36;
    void build_buffers(DevBuf* (&out)[kBuildBufs]) {
        DevBuf* build[kBuildBufs] = {&x, &rec64, &recf, &rad, &keycnt, &keyoff, &keys, &vals, &keys_alt, &vals_alt,
                                     &sort_tmp, &scan_tmp, &rkeys, &rvals, &rkeys_alt, &rvals_alt, &cnt_sorted,
                                     &kept_blk, &kept_off, &kept_mask,
                                     &tile_start, &entry_cnt, &pixC, &ncontrib, &resid, &tile_pairs, &tile_segs,
                                     &tile_real, &tile_real_off, &gv_cnt, &gv_flag, &gv_idx, &gv_segoff, &gv_cursor,
                                     &tile_ck, &pix_stop};
        for (int i = 0; i < kBuildBufs; ++i) out[i] = build[i];
    }
    void release_build_buffers() {
        DevBuf* build[kBuildBufs];
        build_buffers(build);
        for (auto* b : build) b->release();
        compact = true;
    }
    // exchange the build-only buffers with another handle's (a scratch
    // handle of LM_BUILD_COMPACT builds)
    void swap_build_buffers(lm_cache& o) {
        DevBuf* a[kBuildBufs];
        DevBuf* b[kBuildBufs];
        build_buffers(a);
        o.build_buffers(b);
        for (int i = 0; i < kBuildBufs; ++i) a[i]->swap(*b[i]);
    }

    void release_all() {
#define LM_RELEASE_BUF(n) n.release();
        LM_CACHE_BUFFERS(LM_RELEASE_BUF)
#undef LM_RELEASE_BUF
    }
};

namespace {

#define LM_CHECK(cond, code, msg)        \
    do {                                 \
        if (!(cond)) {                   \
            ::lm::set_error(msg);        \
            return code;                 \
        }                                \
    } while (0)

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// Build the cache up to and including the count pass (projection, binning,
// sort, forward render, residuals).  layout: also the per-entry and
// (Gaussian, view) counts and the block layout that the fill pass of a build
// reads (renders and residual norms pass false).
lm_status build_forward(lm_cache* c, const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                        const lm_options* opts, hipStream_t s, bool layout) {
    using namespace lm;
    LM_CHECK(scene && cams && V > 0 && V <= kMaxViews, LM_ERR_INVALID_ARG, "lm_build_cache: bad scene/cameras");
    LM_CHECK(scene->x && scene->N > 0, LM_ERR_INVALID_ARG, "lm_build_cache: empty scene");
    LM_CHECK(scene->sh_degree >= 0 && scene->sh_degree <= 3, LM_ERR_INVALID_ARG, "sh_degree must be 0..3");
    int TW = 16, TH = 16, dtype = LM_CACHE_F32, thin = 0;
    if (opts) {
        if (opts->tile_w > 0) TW = opts->tile_w;
        if (opts->tile_h > 0) TH = opts->tile_h;
        dtype = opts->cache_dtype;
        thin = opts->thin_window;
    }
    LM_CHECK(thin >= 0 && thin <= LM_THIN_WINDOW_MAX, LM_ERR_INVALID_ARG, "thin_window must be 0..4096");
    LM_CHECK(thin == 0 || dtype == LM_CACHE_F32, LM_ERR_UNSUPPORTED,
             "a thinned cache stores no pair values: cache_dtype must be LM_CACHE_F32");
    LM_CHECK(TW * TH <= kMaxTilePix && TW > 0 && TH > 0, LM_ERR_INVALID_ARG, "tile_w * tile_h must be 1..256");
    LM_CHECK((TW & (TW - 1)) == 0, LM_ERR_INVALID_ARG, "tile_w must be a power of two");
    LM_CHECK(dtype == LM_CACHE_F32 || dtype == LM_CACHE_BF16 || dtype == LM_CACHE_F16, LM_ERR_INVALID_ARG,
             "cache_dtype must be LM_CACHE_F32, _BF16 or _F16");
    // record ids are 32-bit, and one-thread-per-record launches must stay
    // below 2^32 work-items after rounding up to whole workgroups
    LM_CHECK(scene->N * (int64_t)V < ((int64_t)1 << 32) - 65536, LM_ERR_CAPACITY, "N * V must fit in 32 bits");
    c->built = false;
    c->gram_valid = false;
    c->bj_valid = false;
    c->compact = false;
    c->weighted = false;
    c->N = scene->N;
    c->deg = scene->sh_degree;
    c->P = 11 + 3 * (c->deg + 1) * (c->deg + 1);
    c->V = V;
    c->TW = TW;
    c->TH = TH;
    c->dtype = dtype;
    c->thin_k = thin;
    c->cams_h.resize(V);
    int64_t tile_base = 0, pix_base = 0;
    std::vector<int32_t> tv;
    for (int v = 0; v < V; ++v) {
        const lm_camera& in = cams[v];
        LM_CHECK(in.W > 0 && in.H > 0, LM_ERR_INVALID_ARG, "camera with empty image");
        CamDev& d = c->cams_h[v];
        for (int i = 0; i < 9; ++i) d.R[i] = in.R[i];
        for (int i = 0; i < 3; ++i) d.t[i] = in.t[i];
        d.fx = in.fx; d.fy = in.fy; d.cx = in.cx; d.cy = in.cy;
        for (int i = 0; i < 3; ++i) d.C[i] = -(d.R[i] * d.t[0] + d.R[3 + i] * d.t[1] + d.R[6 + i] * d.t[2]);
        d.W = in.W; d.H = in.H;
        d.TX = (in.W + TW - 1) / TW;
        d.TY = (in.H + TH - 1) / TH;
        d.tile_base = tile_base;
        d.pix_base = pix_base;
        tv.insert(tv.end(), (size_t)d.TX * d.TY, v);
        tile_base += (int64_t)d.TX * d.TY;
        pix_base += (int64_t)in.W * in.H;
    }
    c->n_tiles = tile_base;
    c->n_pix = pix_base;
    LM_CHECK(c->n_tiles < ((int64_t)1 << 32), LM_ERR_CAPACITY, "too many tiles");
    const int64_t N = c->N, R = N * (int64_t)V, P = c->P;
    LM_HIP(c->cams.ensure(sizeof(CamDev) * V));
    LM_HIP(hipMemcpyAsync(c->cams.p, c->cams_h.data(), sizeof(CamDev) * V, hipMemcpyHostToDevice, s));
    LM_HIP(c->tile_view.ensure(sizeof(int32_t) * c->n_tiles));
    LM_HIP(hipMemcpyAsync(c->tile_view.p, tv.data(), sizeof(int32_t) * c->n_tiles, hipMemcpyHostToDevice, s));
    LM_HIP(c->x.ensure(sizeof(float) * P * N));
    LM_HIP(hipMemcpyAsync(c->x.p, scene->x, sizeof(float) * P * N, hipMemcpyDeviceToDevice, s));

    // projection and key counts
    LM_HIP(c->rec64.ensure(sizeof(double) * lm::kRecStride * R));
    LM_HIP(c->recf.ensure(sizeof(float) * 3 * R));
    LM_HIP(c->rad.ensure(sizeof(int32_t) * R));
    LM_HIP(c->keycnt.ensure(sizeof(uint32_t) * R));
    LM_HIP(c->keyoff.ensure(sizeof(uint64_t) * (R + 1)));
    LM_HIP(c->scan_tmp.ensure(std::max(scan_tmp_bytes(R), scan_tmp_bytes(N * (int64_t)V + 1)) + 1024));
    { LM_PROF("project", s);
    LM_HIP(launch_project(c->cams.as<CamDev>(), c->x.as<float>(), N, V, c->deg, TW, TH, c->rec64.as<double>(),
                          c->recf.as<float>(), c->rad.as<int32_t>(), c->keycnt.as<uint32_t>(), s)); }

    // depth sort of the records of every view (stable: ties keep the id order)
    int view_bits = 0;
    while ((1 << view_bits) < V) ++view_bits;
    LM_HIP(c->rkeys.ensure(sizeof(uint64_t) * R));
    LM_HIP(c->rkeys_alt.ensure(sizeof(uint64_t) * R));
    LM_HIP(c->rvals.ensure(sizeof(uint32_t) * R));
    LM_HIP(c->rvals_alt.ensure(sizeof(uint32_t) * R));
    LM_HIP(c->cnt_sorted.ensure(sizeof(uint32_t) * R));
    LM_HIP(c->sort_tmp.ensure(radix_tmp_bytes(R)));
    const uint32_t* order = nullptr;
    { LM_PROF("depth_sort", s);
    LM_HIP(launch_record_keys(c->recf.as<float>(), c->keycnt.as<uint32_t>(), N, V, c->rkeys.as<uint64_t>(),
                              c->rvals.as<uint32_t>(), s));
    bool ralt = false;
    LM_HIP(radix_sort_pairs(c->rkeys.as<uint64_t>(), c->rvals.as<uint32_t>(), c->rkeys_alt.as<uint64_t>(),
                            c->rvals_alt.as<uint32_t>(), R, 0, 31 + view_bits, c->sort_tmp.p, c->sort_tmp.cap,
                            &ralt, s));
    order = ralt ? c->rvals_alt.as<uint32_t>() : c->rvals.as<uint32_t>();
    LM_HIP(launch_gather_counts(order, c->keycnt.as<uint32_t>(), R, c->cnt_sorted.as<uint32_t>(), s));
    LM_HIP(exclusive_scan_u32_to_u64(c->cnt_sorted.as<uint32_t>(), c->keyoff.as<uint64_t>(), R, c->scan_tmp.p,
                                     c->scan_tmp.cap, s)); }
    // kept keys per block of records (tiles below a splat's alpha threshold
    // are left out), their offsets, and the total; the tile test's ballots
    // cover every rectangle key
    uint64_t K_rect = 0;
    LM_HIP(hipMemcpyAsync(&K_rect, c->keyoff.as<uint64_t>() + R, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LM_HIP(hipStreamSynchronize(s));
    const int64_t nbk = bin_emit_blocks(R);
    LM_HIP(c->kept_blk.ensure(sizeof(uint32_t) * nbk));
    LM_HIP(c->kept_off.ensure(sizeof(uint64_t) * (nbk + 1)));
    LM_HIP(c->kept_mask.ensure(sizeof(uint64_t) * bin_mask_words((int64_t)K_rect, R)));
    { LM_PROF("bin_emit", s);
    LM_HIP(launch_bin_count(c->cams.as<CamDev>(), N, R, TW, TH, c->recf.as<float>(), c->rad.as<int32_t>(), order,
                            c->keyoff.as<uint64_t>(), c->rec64.as<double>(), c->kept_mask.as<uint64_t>(),
                            c->kept_blk.as<uint32_t>(), s));
    LM_HIP(exclusive_scan_u32_to_u64(c->kept_blk.as<uint32_t>(), c->kept_off.as<uint64_t>(), nbk, c->scan_tmp.p,
                                     c->scan_tmp.cap, s)); }
    uint64_t K = 0;
    LM_HIP(hipMemcpyAsync(&K, c->kept_off.as<uint64_t>() + nbk, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    LM_HIP(hipStreamSynchronize(s));
    c->n_keys = (int64_t)K;
    LM_CHECK(c->n_keys < ((int64_t)1 << 40), LM_ERR_CAPACITY, "too many tile keys");

    // binning in depth order, then a stable sort by tile
    const int64_t Ka = std::max<int64_t>(c->n_keys, 1);
    LM_HIP(c->keys.ensure(sizeof(uint32_t) * Ka));
    LM_HIP(c->vals.ensure(sizeof(uint32_t) * Ka));
    LM_HIP(c->keys_alt.ensure(sizeof(uint32_t) * Ka));
    LM_HIP(c->vals_alt.ensure(sizeof(uint32_t) * Ka));
    LM_HIP(c->sort_tmp.ensure(radix_tmp_bytes(std::max<int64_t>(Ka, R))));
    { LM_PROF("bin_emit", s);
    LM_HIP(launch_bin_emit(c->cams.as<CamDev>(), N, R, TW, TH, c->recf.as<float>(), c->rad.as<int32_t>(), order,
                           c->keyoff.as<uint64_t>(), c->rec64.as<double>(), c->kept_mask.as<uint64_t>(),
                           c->kept_off.as<uint64_t>(), c->n_keys,
                           c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), s)); }
    int tile_bits = 1;
    while (((int64_t)1 << tile_bits) < c->n_tiles) ++tile_bits;
    bool alt = false;
    { LM_PROF("tile_sort", s);
    LM_HIP(radix_sort_pairs_u32(c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), c->keys_alt.as<uint32_t>(),
                                c->vals_alt.as<uint32_t>(), c->n_keys, 0, tile_bits, c->sort_tmp.p,
                                c->sort_tmp.cap, &alt, s)); }
    c->vals_in_alt = alt;
    const uint32_t* skeys = alt ? c->keys_alt.as<uint32_t>() : c->keys.as<uint32_t>();
    LM_HIP(c->tile_start.ensure(sizeof(int64_t) * (c->n_tiles + 1)));
    { LM_PROF("tile_ranges", s); LM_HIP(launch_tile_ranges(skeys, c->n_keys, c->n_tiles, c->tile_start.as<int64_t>(), s)); }

    // forward render and per-entry counts
    LM_HIP(c->entry_cnt.ensure(sizeof(uint32_t) * Ka));
    LM_HIP(c->pixC.ensure(sizeof(double) * 3 * c->n_pix));
    LM_HIP(c->ncontrib.ensure(sizeof(int32_t) * c->n_pix));
    if (layout) LM_HIP(c->pix_stop.ensure(sizeof(uint32_t) * c->n_pix));
    LM_HIP(c->resid.ensure(sizeof(float) * 3 * c->n_pix));
    LM_HIP(c->fsq_part.ensure(sizeof(double) * c->n_tiles));
    LM_HIP(c->tile_pairs.ensure(sizeof(uint32_t) * c->n_tiles));
    LM_HIP(c->tile_blk.ensure(sizeof(uint32_t) * lm::kTileBlocks * std::max<int64_t>(c->n_tiles, 1)));
    LM_HIP(c->tile_segs.ensure(sizeof(uint32_t) * c->n_tiles));
    LM_HIP(c->tile_real.ensure(sizeof(uint32_t) * c->n_tiles));
    LM_HIP(c->gv_cnt.ensure(sizeof(uint32_t) * (R + 1)));
    LM_HIP(hipMemsetAsync(c->gv_cnt.p, 0, sizeof(uint32_t) * (R + 1), s));
    if (thin) LM_HIP(c->tile_ck.ensure(sizeof(uint32_t) * std::max<int64_t>(c->n_tiles, 1)));
    RasterArgs ra{};
    ra.cams = c->cams.as<CamDev>();
    ra.tile_view = c->tile_view.as<int32_t>();
    ra.tile_start = c->tile_start.as<int64_t>();
    ra.vals = c->sorted_vals();
    ra.rec64 = c->rec64.as<double>();
    ra.N = N; ra.V = V; ra.TW = TW; ra.TH = TH;
    ra.layout = layout ? 1 : 0;
    ra.target = target;
    ra.entry_cnt = c->entry_cnt.as<uint32_t>();
    ra.pixC = c->pixC.as<double>();
    ra.ncontrib = c->ncontrib.as<int32_t>();
    ra.pix_stop = layout ? c->pix_stop.as<uint32_t>() : nullptr;
    ra.resid = c->resid.as<float>();
    ra.fsq_part = c->fsq_part.as<double>();
    ra.tile_pairs = c->tile_pairs.as<uint32_t>();
    ra.tile_blk = c->tile_blk.as<uint32_t>();
    ra.tile_segs = c->tile_segs.as<uint32_t>();
    ra.tile_real = c->tile_real.as<uint32_t>();
    ra.gv_cnt = c->gv_cnt.as<uint32_t>();
    ra.n_pix = c->n_pix;
    ra.thin_k = thin;
    ra.tile_ck = c->tile_ck.as<uint32_t>();
    { LM_PROF("raster_count", s); LM_HIP(launch_raster(false, dtype, c->n_tiles, ra, s)); }
    return LM_OK;
}

lm_status build_fill(lm_cache* c, hipStream_t s) {
    using namespace lm;
    const int64_t N = c->N, V = c->V, NV = N * V;
    LM_HIP(c->tile_pair_off.ensure(sizeof(uint64_t) * (c->n_tiles + 1)));
    LM_HIP(c->tile_seg_off.ensure(sizeof(uint64_t) * (c->n_tiles + 1)));
    LM_HIP(c->tile_real_off.ensure(sizeof(uint64_t) * (c->n_tiles + 1)));
    LM_HIP(c->scan_tmp.ensure(std::max(scan_tmp_bytes(c->n_tiles), scan_tmp_bytes(NV)) + 1024));
    LM_HIP(exclusive_scan_u32_to_u64(c->tile_pairs.as<uint32_t>(), c->tile_pair_off.as<uint64_t>(), c->n_tiles,
                                     c->scan_tmp.p, c->scan_tmp.cap, s));
    LM_HIP(exclusive_scan_u32_to_u64(c->tile_segs.as<uint32_t>(), c->tile_seg_off.as<uint64_t>(), c->n_tiles,
                                     c->scan_tmp.p, c->scan_tmp.cap, s));
    LM_HIP(exclusive_scan_u32_to_u64(c->tile_real.as<uint32_t>(), c->tile_real_off.as<uint64_t>(), c->n_tiles,
                                     c->scan_tmp.p, c->scan_tmp.cap, s));
    LM_HIP(c->gv_flag.ensure(sizeof(uint32_t) * NV));
    LM_HIP(c->gv_idx.ensure(sizeof(uint64_t) * (NV + 1)));
    LM_HIP(c->gv_segoff.ensure(sizeof(uint64_t) * (NV + 1)));
    LM_HIP(launch_flag_nonzero(c->gv_cnt.as<uint32_t>(), NV, c->gv_flag.as<uint32_t>(), s));
    LM_HIP(exclusive_scan_u32_to_u64(c->gv_flag.as<uint32_t>(), c->gv_idx.as<uint64_t>(), NV, c->scan_tmp.p,
                                     c->scan_tmp.cap, s));
    LM_HIP(exclusive_scan_u32_to_u64(c->gv_cnt.as<uint32_t>(), c->gv_segoff.as<uint64_t>(), NV, c->scan_tmp.p,
                                     c->scan_tmp.cap, s));
    uint64_t host3[4] = {0, 0, 0, 0};
    LM_HIP(hipMemcpyAsync(&host3[0], c->tile_pair_off.as<uint64_t>() + c->n_tiles, 8, hipMemcpyDeviceToHost, s));
    LM_HIP(hipMemcpyAsync(&host3[1], c->tile_seg_off.as<uint64_t>() + c->n_tiles, 8, hipMemcpyDeviceToHost, s));
    LM_HIP(hipMemcpyAsync(&host3[2], c->gv_idx.as<uint64_t>() + NV, 8, hipMemcpyDeviceToHost, s));
    LM_HIP(hipMemcpyAsync(&host3[3], c->tile_real_off.as<uint64_t>() + c->n_tiles, 8, hipMemcpyDeviceToHost, s));
    LM_HIP(hipStreamSynchronize(s));
    c->n_slots = c->thin_k ? 0 : (int64_t)host3[0];
    c->n_pieces = c->thin_k ? (int64_t)host3[0] : 0;
    c->n_pairs = (int64_t)host3[3];
    c->n_seg = (int64_t)host3[1];
    c->n_gv = (int64_t)host3[2];
    LM_CHECK(c->n_seg < ((int64_t)1 << 32) - 65536 && c->n_gv < ((int64_t)1 << 32) - 65536, LM_ERR_CAPACITY,
             "segment or (Gaussian, view) count exceeds 32 bits");
    const int64_t nseg_a = std::max<int64_t>(c->n_seg, 1), ngv_a = std::max<int64_t>(c->n_gv, 1);
    LM_HIP(c->gv_rec.ensure(sizeof(uint32_t) * ngv_a));
    LM_HIP(c->gv_seg_off.ensure(sizeof(uint32_t) * (ngv_a + 1)));
    LM_HIP(c->gv_first.ensure(sizeof(uint32_t) * (N + 1)));
    LM_HIP(c->gv_cursor.ensure(sizeof(uint32_t) * ngv_a));
    LM_HIP(hipMemsetAsync(c->gv_cursor.p, 0, sizeof(uint32_t) * ngv_a, s));
    LM_HIP(c->gv_segs.ensure(sizeof(uint32_t) * nseg_a));
    LM_HIP(c->seg_pos.ensure(sizeof(uint32_t) * nseg_a));
    LM_HIP(c->list_gv.ensure(sizeof(uint32_t) * nseg_a));
    LM_HIP(launch_gv_compact(c->gv_cnt.as<uint32_t>(), c->gv_idx.as<uint64_t>(), c->gv_segoff.as<uint64_t>(), N,
                             (int)V, c->gv_rec.as<uint32_t>(), c->gv_seg_off.as<uint32_t>(),
                             c->gv_first.as<uint32_t>(), s));
    c->seg_stride = round_up(nseg_a, 8);
    if (c->thin_k) {
        // thinned cache: pieces and per-pixel checkpoints instead of pair planes
        LM_HIP(c->tile_ck_off.ensure(sizeof(uint64_t) * (c->n_tiles + 1)));
        LM_HIP(exclusive_scan_u32_to_u64(c->tile_ck.as<uint32_t>(), c->tile_ck_off.as<uint64_t>(), c->n_tiles,
                                         c->scan_tmp.p, c->scan_tmp.cap, s));
        uint64_t nck = 0;
        LM_HIP(hipMemcpyAsync(&nck, c->tile_ck_off.as<uint64_t>() + c->n_tiles, 8, hipMemcpyDeviceToHost, s));
        LM_HIP(hipStreamSynchronize(s));
        c->n_ck = (int64_t)nck;
        const int64_t np_a = std::max<int64_t>(c->n_pieces, 1);
        LM_HIP(c->piece_seg.ensure(sizeof(uint32_t) * np_a));
        LM_HIP(c->piece_mask.ensure(sizeof(uint64_t) * np_a));
        LM_HIP(c->piece_cmask.ensure(sizeof(uint64_t) * np_a));
        LM_HIP(c->pix_ck.ensure(sizeof(uint32_t) * std::max<int64_t>(c->n_pix, 1)));
        // two spare entries: a walk may read one past a pixel's last checkpoint
        LM_HIP(c->ck.ensure(sizeof(float) * 4 * (c->n_ck + 2)));
        LM_HIP(hipMemsetAsync(c->ck.as<float>() + 4 * c->n_ck, 0, sizeof(float) * 8, s));
        c->pT.release();
        c->pD.release();
        c->ppix.release();
        c->run_seg.release();
        c->pair_stride = 8;
    } else {
    // pair and segment arrays (planes padded so 8-wide vector loads stay inside);
    // the zero fill doubles as the padding of every segment to a multiple of 8
    c->pair_stride = round_up(c->n_slots, 8) + 8;
    const size_t wb = dtype_bytes(c->dtype);
    LM_HIP(c->pT.ensure(wb * c->pair_stride));
    LM_HIP(c->pD.ensure(wb * 3 * c->pair_stride));
    LM_HIP(c->ppix.ensure(c->pair_stride));
    // the fill pass writes every slot of every segment (pairs and padding);
    // only the slots past the last segment are cleared here
    if (c->pair_stride > c->n_slots) {
        const size_t tail = (size_t)(c->pair_stride - c->n_slots);
        LM_HIP(hipMemsetAsync((char*)c->pT.p + wb * c->n_slots, 0, wb * tail, s));
        for (int ch = 0; ch < 3; ++ch)
            LM_HIP(hipMemsetAsync((char*)c->pD.p + wb * (ch * c->pair_stride + c->n_slots), 0, wb * tail, s));
        LM_HIP(hipMemsetAsync(c->ppix.as<uint8_t>() + c->n_slots, 0, tail, s));
    }
    LM_HIP(c->run_seg.ensure(sizeof(uint32_t) * (c->pair_stride / 8)));
    }
    LM_HIP(c->seg_gv.ensure(sizeof(uint32_t) * nseg_a));
    LM_HIP(c->seg_f.ensure(sizeof(float) * (c->thin_k ? 9 : 6) * c->seg_stride));
    RasterArgs ra{};
    ra.cams = c->cams.as<CamDev>();
    ra.tile_view = c->tile_view.as<int32_t>();
    ra.tile_start = c->tile_start.as<int64_t>();
    ra.vals = c->sorted_vals();
    ra.rec64 = c->rec64.as<double>();
    ra.N = N; ra.V = (int)V; ra.TW = c->TW; ra.TH = c->TH;
    ra.entry_cnt = c->entry_cnt.as<uint32_t>();
    ra.pixC = c->pixC.as<double>();
    ra.n_pix = c->n_pix;
    ra.tile_pair_off = c->tile_pair_off.as<int64_t>();
    ra.tile_seg_off = c->tile_seg_off.as<int64_t>();
    ra.gv_idx = c->gv_idx.as<uint64_t>();
    ra.gv_segoff = c->gv_segoff.as<uint64_t>();
    ra.gv_cursor = c->gv_cursor.as<uint32_t>();
    ra.gv_segs = c->gv_segs.as<uint32_t>();
    ra.pT = c->pT.p;
    ra.pD = c->pD.p;
    ra.pair_stride = c->pair_stride;
    ra.ppix = c->ppix.as<uint8_t>();
    ra.seg_gv = c->seg_gv.as<uint32_t>();
    ra.tile_blk = c->tile_blk.as<uint32_t>();
    ra.seg_f = c->seg_f.as<float>();
    ra.seg_stride = c->seg_stride;
    ra.run_seg = c->run_seg.as<uint32_t>();
    ra.thin_k = c->thin_k;
    ra.ncontrib = c->ncontrib.as<int32_t>();
    ra.pix_stop = c->pix_stop.as<uint32_t>();
    ra.tile_ck_off = c->tile_ck_off.as<int64_t>();
    ra.pix_ck = c->pix_ck.as<uint32_t>();
    ra.ck = c->ck.as<float>();
    ra.piece_seg = c->piece_seg.as<uint32_t>();
    ra.piece_mask = c->piece_mask.as<uint64_t>();
    ra.piece_cmask = c->piece_cmask.as<uint64_t>();
    { LM_PROF("raster_fill", s); LM_HIP(launch_raster(true, c->dtype, c->n_tiles, ra, s)); }
    { LM_PROF("gv_sort", s); LM_HIP(launch_gv_sort(c->gv_seg_off.as<uint32_t>(), c->n_gv, c->gv_segs.as<uint32_t>(), s));
      LM_HIP(launch_seg_pos(c->gv_segs.as<uint32_t>(), c->seg_gv.as<uint32_t>(), c->n_seg, c->seg_pos.as<uint32_t>(),
                            c->list_gv.as<uint32_t>(), s)); }
    // linearised projection of every (Gaussian, view) at x
    c->lin_stride = round_up(ngv_a, 8);
    LM_HIP(c->lin.ensure(sizeof(float) * lm::kLin * c->lin_stride));
    { LM_PROF("linearize", s); LM_HIP(launch_linearize(c->view(), c->x.as<float>(), c->lin.as<float>(), s)); }
    // product workspaces
    LM_HIP(c->dyc.ensure(sizeof(float) * 9 * ngv_a));
    LM_HIP(c->gmom.ensure(sizeof(float) * 9 * nseg_a));
    const int64_t nwav = lm::gv_reduce_waves(nseg_a);
    LM_HIP(c->gvsum.ensure(sizeof(float) * 9 * ngv_a));
    LM_HIP(c->gvchain.ensure((sizeof(double) * 11 + sizeof(float) * 3 * (c->deg + 1) * (c->deg + 1)) * c->lin_stride));
    LM_HIP(c->edge_m.ensure(sizeof(float) * 2 * 9 * nwav));
    LM_HIP(c->ekey_m.ensure(sizeof(uint32_t) * nwav));
    LM_HIP(c->jp_part.ensure(sizeof(double) * c->n_tiles));
    LM_HIP(c->pg_part.ensure(sizeof(double) * (chain_blocks(N) + 1)));
    LM_HIP(c->scalar.ensure(sizeof(double) * 4));
    c->built = true;
    return LM_OK;
}

lm::ApplyBatch batch_of(lm_cache* const* cs, int n) {
    lm::ApplyBatch B{};
    B.n = n;
    B.scale = 1.0f;
    B.tile_off[0] = 0;
    for (int i = 0; i < n; ++i) {
        B.a[i] = cs[i]->apply_args();
        B.tile_off[i + 1] = B.tile_off[i] + cs[i]->n_tiles;
    }
    return B;
}

lm_status apply_JT_internal(const lm_cache* c, const float* u, float scale, float* g, hipStream_t s) {
    lm_cache* cm = const_cast<lm_cache*>(c);
    lm::ApplyBatch B = batch_of(&cm, 1);
    B.a[0].uin = u;
    B.a[0].out = g;
    B.scale = scale;
    { LM_PROF("apply_tile_JT", s); LM_HIP(lm::launch_apply_tile(2, B, s)); }
    { LM_PROF("gv_reduce", s); LM_HIP(lm::launch_gv_reduce_moments(B, s)); }
    { LM_PROF("chain", s); LM_HIP(lm::launch_chain(B, s)); }
    return LM_OK;
}

// g_i = J_i^T J_i p_i + lambda M_i p_i for every subset of the batch
lm_status apply_JtJ_batch(const lm::ApplyBatch& B, hipStream_t s) {
    { LM_PROF("tangent", s); LM_HIP(lm::launch_tangent(B, s)); }
    { LM_PROF("apply_tile_JtJ", s); LM_HIP(lm::launch_apply_tile(3, B, s)); }
    { LM_PROF("gv_reduce", s); LM_HIP(lm::launch_gv_reduce_moments(B, s)); }
    { LM_PROF("chain", s); LM_HIP(lm::launch_chain(B, s)); }
    return LM_OK;
}

lm_status apply_JtJ_internal(lm_cache* c, const float* p, float lambda, const float* M, float diag_floor, float* g,
                             double* pg_part, const int32_t* stop, hipStream_t s) {
    lm::ApplyBatch B = batch_of(&c, 1);
    B.a[0].p = p;
    B.a[0].stop = stop;
    B.a[0].M = M;
    B.a[0].out = g;
    B.a[0].pg_part = pg_part;
    B.lambda = lambda;
    B.diag_floor = diag_floor;
    return apply_JtJ_batch(B, s);
}

// Non-blocking stream (default priority) that the iteration is captured
// into; the graph itself is launched on the caller's stream.
hipError_t capture_stream(hipStream_t* out) {
    static hipStream_t cs[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!cs[dev]) {
        e = hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = cs[dev];
    return hipSuccess;
}

// The objective's terms for the V views of an image-layout pair (a, t):
// a is the image, or the residual image - t when add_target.  Partial sums
// of E stay in ws->obj_part; E_total and E_view (dev, may be null) receive
// the total and the per-view sums (E_view needs cams_dev).
lm_status objective_check(const lm_objective* o) {
    LM_CHECK(o, LM_ERR_INVALID_ARG, "objective is NULL");
    LM_CHECK(o->kind == LM_OBJ_L2 || o->kind == LM_OBJ_L1_SSIM, LM_ERR_INVALID_ARG,
             "objective kind must be LM_OBJ_L2 or LM_OBJ_L1_SSIM");
    LM_CHECK(o->kind == LM_OBJ_L2 || (o->eps > 0.0f && o->lambda1 >= 0.0f && o->lambda2 >= 0.0f),
             LM_ERR_INVALID_ARG, "objective needs eps > 0 and lambda1, lambda2 >= 0");
    return LM_OK;
}

lm_status run_objective(lm_cache* ws, const float* a, const float* t, bool add_target, const std::vector<int>& Ws,
                        const std::vector<int>& Hs, const lm_objective* o, float* w, float* e, double* E_total,
                        const lm::CamDev* cams_dev, double* E_view, hipStream_t s) {
    const int V = (int)Ws.size();
    int64_t nparts = 0;
    std::vector<int64_t> p0(V);
    for (int v = 0; v < V; ++v) {
        p0[v] = nparts;
        nparts += lm::objective_blocks(Ws[v], Hs[v]);
    }
    LM_HIP(ws->obj_part.ensure(sizeof(double) * std::max<int64_t>(nparts, 1)));
    lm::ObjectiveArgs A{};
    A.a = a;
    A.t = t;
    A.w = w;
    A.e = e;
    A.part = ws->obj_part.as<double>();
    A.kind = o->kind;
    A.add_target = add_target ? 1 : 0;
    A.lam1 = o->lambda1;
    A.lam2 = o->lambda2;
    A.eps = o->eps;
    lm::objective_window(A.g);
    int64_t off = 0;
    for (int v = 0; v < V; ++v) {
        A.off = off;
        A.part0 = p0[v];
        A.W = Ws[v];
        A.H = Hs[v];
        LM_HIP(lm::launch_objective(A, s));
        off += 3 * (int64_t)Ws[v] * Hs[v];
    }
    if (E_total) LM_HIP(lm::reduce_f64(ws->obj_part.as<double>(), nparts, E_total, s));
    if (E_view) LM_HIP(lm::launch_objective_view_sums(cams_dev, V, ws->obj_part.as<double>(), E_view, s));
    return LM_OK;
}

// Binds a handle to the context of the running entry point; the context
// counts its handles so that it is not destroyed under them.
void bind_ctx(lm_cache* c) {
    lm_ctx* x = lm::g_ctx;
    if (c->ctx == x) return;
    if (c->ctx) --c->ctx->n_caches;
    c->ctx = x;
    ++x->n_caches;
}

void free_handle(lm_cache* c) {
    if (c->ctx) --c->ctx->n_caches;
    c->release_all();
    delete c;
}

}  // namespace

extern "C" {

const char* lm_last_error(void) { return lm::g_last_error.c_str(); }

lm_status lm_ctx_create(const lm_allocator* allocator, lm_ctx** out) {
    LM_CHECK(out, LM_ERR_INVALID_ARG, "lm_ctx_create: out is NULL");
    LM_CHECK(!allocator || (allocator->alloc && allocator->free), LM_ERR_INVALID_ARG,
             "lm_ctx_create: alloc and free are both required");
    lm_ctx* x = new (std::nothrow) lm_ctx();
    LM_CHECK(x, LM_ERR_HIP, "out of host memory");
    if (allocator) x->al = *allocator;
    *out = x;
    return LM_OK;
}

lm_status lm_ctx_destroy(lm_ctx* ctx) {
    if (!ctx) return LM_OK;
    LM_CHECK(ctx != &lm::g_default_ctx, LM_ERR_INVALID_ARG, "lm_ctx_destroy: the default context");
    LM_CHECK(ctx->n_caches == 0, LM_ERR_INVALID_ARG, "lm_ctx_destroy: caches of the context are still alive");
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    if (ctx->part || ctx->persist_dev) (void)hipDeviceSynchronize();
    if (ctx->part) {
        if (ctx->part_al.alloc) ctx->part_al.free(ctx->part_al.user, ctx->part, (void*)ctx->part_stream);
        else (void)hipFree(ctx->part);
    }
    if (ctx->persist_exec) (void)hipGraphExecDestroy(ctx->persist_exec);
    if (ctx->persist_dev) {
        if (ctx->persist_al.alloc) ctx->persist_al.free(ctx->persist_al.user, ctx->persist_dev, (void*)ctx->persist_stream);
        else (void)hipFree(ctx->persist_dev);
    }
    delete ctx;
    return LM_OK;
}

lm_status lm_vec_dot(lm_ctx* ctx, const float* a, const float* b, int64_t n, double* out, void* stream) {
    lm_ctx* x = ctx ? ctx : &lm::g_default_ctx;
    lm::StreamScope lm_stream_scope_(S(stream), x);
    LM_CHECK(((a && b) || n == 0) && out && n >= 0, LM_ERR_INVALID_ARG, "lm_vec_dot: bad argument");
    hipStream_t s = S(stream);
    const size_t need = sizeof(double) * (size_t)lm::dot_partial_count(n);
    if (x->part_cap < need) {
        if (x->part) {
            LM_HIP(hipStreamSynchronize(s));
            if (x->part_al.alloc) x->part_al.free(x->part_al.user, x->part, (void*)x->part_stream);
            else LM_HIP(hipFree(x->part));
            x->part = nullptr;
            x->part_cap = 0;
        }
        if (x->al.alloc) {
            x->part = x->al.alloc(x->al.user, need, (void*)s);
            LM_CHECK(x->part, LM_ERR_HIP, "lm_vec_dot: allocation failed");
        } else {
            LM_HIP(hipMalloc(&x->part, need));
        }
        x->part_cap = need;
        x->part_al = x->al;
        x->part_stream = s;
    }
    LM_HIP(lm::launch_dot(a, b, n, (double*)x->part, out, s));
    return LM_OK;
}

lm_status lm_vec_dot_static(const float* a, const float* b, int64_t n, double* out, void* stream) {
    LM_CHECK(((a && b) || n == 0) && out && n >= 0, LM_ERR_INVALID_ARG, "lm_vec_dot_static: bad argument");
    LM_CHECK(n <= LM_VEC_DOT_STATIC_MAX_N, LM_ERR_CAPACITY,
             "lm_vec_dot_static: n exceeds the maximum of 2^40 elements");
    LM_CHECK(lm::dot_partial_count(n) <= lm::dot_static_capacity(), LM_ERR_CAPACITY,
             "lm_vec_dot_static: partial sums exceed the static scratch");
    double* part = nullptr;
    LM_HIP(lm::dot_static_scratch(&part));
    LM_HIP(lm::launch_dot(a, b, n, part, out, S(stream)));
    return LM_OK;
}

lm_status lm_vec_axpy(const float* x, const float* d, float gamma, int64_t n, float* out, void* stream) {
    LM_CHECK((x && d && out) || n == 0, LM_ERR_INVALID_ARG, "lm_vec_axpy: bad argument");
    LM_CHECK(n >= 0, LM_ERR_INVALID_ARG, "lm_vec_axpy: bad argument");
    LM_HIP(lm::launch_axpy(x, d, gamma, n, out, S(stream)));
    return LM_OK;
}

lm_status lm_build_cache(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                         const lm_options* opts, void* stream, lm_cache** inout, float* b, double* F_sqnorm) {
    lm::StreamScope lm_stream_scope_(S(stream), opts ? opts->ctx : nullptr);
    LM_CHECK(inout, LM_ERR_INVALID_ARG, "lm_build_cache: inout is NULL");
    LM_CHECK(target, LM_ERR_INVALID_ARG, "lm_build_cache: target is NULL");
    lm::set_error("");
    lm_cache* c = *inout;
    bool created = false;
    if (!c) {
        c = new (std::nothrow) lm_cache();
        LM_CHECK(c, LM_ERR_HIP, "out of host memory");
        created = true;
    }
    bind_ctx(c);
    hipStream_t s = S(stream);
    // a compact build with a scratch handle borrows its build-only buffers
    lm_cache* scratch = nullptr;
    if (opts && (opts->flags & LM_BUILD_COMPACT) && opts->scratch) {
        if (!*opts->scratch) {
            *opts->scratch = new (std::nothrow) lm_cache();
            if (!*opts->scratch) {
                if (created) free_handle(c);
                LM_CHECK(false, LM_ERR_HIP, "out of host memory");
            }
        }
        scratch = *opts->scratch;
        bind_ctx(scratch);
        LM_CHECK(scratch != c, LM_ERR_INVALID_ARG, "lm_build_cache: the scratch handle is the cache itself");
        c->swap_build_buffers(*scratch);
    }
    lm_status st = build_forward(c, scene, cams, V, target, opts, s, true);
    if (st == LM_OK) st = build_fill(c, s);
    if (st == LM_OK && F_sqnorm) {
        hipError_t e = lm::reduce_f64(c->fsq_part.as<double>(), c->n_tiles, F_sqnorm, s);
        if (e != hipSuccess) {
            lm::set_error(std::string("reduce: ") + hipGetErrorString(e));
            st = LM_ERR_HIP;
        }
    }
    if (st == LM_OK && b) st = apply_JT_internal(c, c->resid.as<float>(), -1.0f, b, s);
    if (scratch) {
        // the build is enqueued; the scratch handle takes its buffers back
        // (later work on them is ordered on the stream)
        c->swap_build_buffers(*scratch);
    }
    if (st == LM_OK && opts && (opts->flags & LM_BUILD_COMPACT)) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            lm::set_error(std::string("lm_build_cache: ") + hipGetErrorString(e));
            st = LM_ERR_HIP;
        } else {
            c->release_build_buffers();
        }
    }
    if (st != LM_OK) {
        if (created) free_handle(c);
        return st;
    }
    *inout = c;
    return LM_OK;
}

lm_status lm_cache_destroy(lm_cache* cache) {
    if (!cache) return LM_OK;
    (void)hipDeviceSynchronize();
    free_handle(cache);
    return LM_OK;
}

lm_status lm_cache_get_info(const lm_cache* c, lm_cache_info* info) {
    LM_CHECK(c && info, LM_ERR_INVALID_ARG, "lm_cache_get_info: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    memset(info, 0, sizeof(*info));
    info->N = c->N;
    info->n_keys = c->n_keys;
    info->n_pairs = c->n_pairs;
    info->n_pair_slots = c->n_slots;
    info->n_segments = c->n_seg;
    info->n_gv = c->n_gv;
    info->n_pixels = c->n_pix;
    info->n_tiles = c->n_tiles;
    const int64_t wb = (int64_t)lm::dtype_bytes(c->dtype);
    info->cache_bytes = c->thin_k
                            ? c->n_pieces * (4 + 8 + 8) + c->n_ck * 16 + c->n_pix * 4 + c->n_tiles * 8 +
                                  c->n_seg * (4 + 4 + 36)
                            : c->n_slots * (4 * wb + 1) + (c->n_slots / 8) * 4 + c->n_seg * (4 + 4 + 24);
    info->thin_window = c->thin_k;
    info->n_pieces = c->n_pieces;
    info->n_checkpoints = c->n_ck;
    info->device_bytes = (int64_t)c->device_bytes();
    info->V = c->V;
    info->P = c->P;
    info->tile_w = c->TW;
    info->tile_h = c->TH;
    info->cache_dtype = c->dtype;
    info->sh_degree = c->deg;
    return LM_OK;
}

lm_status lm_cache_memory(const lm_cache* c, lm_buffer_bytes* out, int32_t capacity, int32_t* n) {
    LM_CHECK(c && n && capacity >= 0 && (out || capacity == 0), LM_ERR_INVALID_ARG, "lm_cache_memory: bad argument");
    int32_t i = 0;
    c->each_buffer([&](const char* name, size_t bytes) {
        if (i < capacity) {
            memset(out[i].name, 0, sizeof(out[i].name));
            strncpy(out[i].name, name, sizeof(out[i].name) - 1);
            out[i].bytes = bytes;
        }
        ++i;
    });
    *n = i;
    return LM_OK;
}

// The per-(Gaussian, view) Gram values of the current build, computed on
// first use; every quantity derived from J^T J per Gaussian reads them.
static lm_status ensure_gram(lm_cache* cm, hipStream_t s) {
    if (cm->gram_valid) return LM_OK;
    constexpr int64_t kG = lm::kGramValues;
    const int64_t nseg_a = std::max<int64_t>(cm->n_seg, 1);
    const int64_t nwav = lm::gv_reduce_waves(nseg_a);
    LM_HIP(cm->gram.ensure(sizeof(float) * kG * nseg_a));
    LM_HIP(cm->gvgram.ensure(sizeof(float) * kG * std::max<int64_t>(cm->n_gv, 1)));
    LM_HIP(cm->edge_g.ensure(sizeof(float) * 2 * kG * nwav));
    LM_HIP(cm->ekey_g.ensure(sizeof(uint32_t) * nwav));
    LM_HIP(lm::launch_gram(cm->view(), cm->gram.as<float>(), cm->gvgram.as<float>(), cm->edge_g.as<float>(),
                           cm->ekey_g.as<uint32_t>(), s));
    cm->gram_valid = true;
    if (cm->compact) {
        // per-(splat, tile) values: transients of the reduction
        LM_HIP(hipStreamSynchronize(s));
        cm->gram.release();
        cm->edge_g.release();
        cm->ekey_g.release();
    }
    return LM_OK;
}

lm_status lm_cache_trim(lm_cache* c, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c, LM_ERR_INVALID_ARG, "lm_cache_trim: NULL argument");
    LM_HIP(hipStreamSynchronize(S(stream)));
    DevBuf* derived[] = {&c->gram, &c->gvgram, &c->edge_g, &c->ekey_g, &c->coverage, &c->feat_red, &c->tgt_red,
                         &c->bj_L, &c->bj_count};
    for (DevBuf* b : derived) b->release();
    c->gram_valid = false;
    c->bj_valid = false;
    return LM_OK;
}

// Block-Jacobi factors of the current build for (lambda, floor), computed
// on first use (one factorisation per Gaussian from the Gram values).  *n_fallback (host, may be null) receives the number of
// Gaussians whose block did not factor (Jacobi on those).
static lm_status ensure_block_precond(lm_cache* cm, float lambda, float floor_, hipStream_t s,
                                      int32_t* n_fallback) {
    if (cm->bj_valid && cm->bj_lambda == lambda && cm->bj_floor == floor_ && !n_fallback) return LM_OK;
    lm_status st = ensure_gram(cm, s);
    if (st != LM_OK) return st;
    const int64_t N = cm->N, P = cm->P, T = P * (P + 1) / 2;
    LM_HIP(cm->bj_L.ensure(sizeof(float) * T * ((N + 63) / 64) * 64));
    LM_HIP(cm->bj_count.ensure(sizeof(uint32_t)));
    LM_HIP(hipMemsetAsync(cm->bj_count.p, 0, sizeof(uint32_t), s));
    {
        LM_PROF("block_precond", s);
        LM_HIP(lm::launch_bj_factor(cm->view(), cm->gvgram.as<float>(), lambda, floor_, cm->bj_L.as<float>(),
                                    cm->bj_count.as<uint32_t>(), s));
    }
    cm->bj_valid = true;
    cm->bj_lambda = lambda;
    cm->bj_floor = floor_;
    if (n_fallback) {
        uint32_t h = 0;
        LM_HIP(hipMemcpyAsync(&h, cm->bj_count.p, sizeof(h), hipMemcpyDeviceToHost, s));
        LM_HIP(hipStreamSynchronize(s));
        *n_fallback = (int32_t)h;
    }
    return LM_OK;
}

static lm::BlockPrecond block_precond_of(const lm_cache* c) {
    return lm::BlockPrecond{c->bj_L.as<float>(), c->N, c->P};
}

lm_status lm_jacobi_diag(const lm_cache* c, float* M, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && M, LM_ERR_INVALID_ARG, "lm_jacobi_diag: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    LM_PROF("jacobi_diag", S(stream));
    lm_status st = ensure_gram(cm, S(stream));
    if (st != LM_OK) return st;
    // the chain's per-(Gaussian, view) workspace (11 doubles per record
    // first) serves as the diagonal's scratch: no product runs meanwhile
    LM_HIP(lm::launch_jacobi_diag(c->view(), cm->gvgram.as<float>(), cm->gvchain.as<double>(), M, S(stream)));
    return LM_OK;
}

lm_status lm_pair_coverage(const lm_cache* c, float* coverage, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && coverage, LM_ERR_INVALID_ARG, "lm_pair_coverage: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    lm_status st = ensure_gram(cm, S(stream));
    if (st != LM_OK) return st;
    LM_HIP(lm::launch_coverage(c->view(), cm->gvgram.as<float>(), coverage, S(stream)));
    return LM_OK;
}

lm_status lm_block_jacobi(const lm_cache* c, const int64_t* gaussians, int64_t n, float* blocks, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && (n == 0 || (gaussians && blocks)) && n >= 0, LM_ERR_INVALID_ARG, "lm_block_jacobi: bad argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    if (n == 0) return LM_OK;
    lm_status st = ensure_gram(cm, S(stream));
    if (st != LM_OK) return st;
    LM_HIP(lm::launch_block_rows(c->view(), cm->gvgram.as<float>(), gaussians, n, 0, 0.0f, 0.0f, blocks, nullptr,
                                 S(stream)));
    return LM_OK;
}

lm_status lm_precond_targets(const lm_cache* c, float lambda, float diag_floor, float shrink, float* t, float* mask,
                             void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && t && mask, LM_ERR_INVALID_ARG, "lm_precond_targets: NULL argument");
    LM_CHECK(lambda >= 0.0f && diag_floor >= 0.0f, LM_ERR_INVALID_ARG, "lambda and diag_floor must be >= 0");
    LM_CHECK(shrink >= 0.0f && shrink <= 1.0f, LM_ERR_INVALID_ARG, "shrink must be in [0, 1]");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    LM_PROF("precond_targets", S(stream));
    lm_status st = ensure_gram(cm, S(stream));
    if (st != LM_OK) return st;
    LM_HIP(lm::launch_block_rows(c->view(), cm->gvgram.as<float>(), nullptr, 0, 1, lambda, diag_floor, t, mask,
                                 S(stream)));
    if (shrink != 1.0f) {
        LM_HIP(cm->tgt_red.ensure(sizeof(double) * lm::shrink_scratch_doubles(c->P)));
        LM_HIP(lm::launch_target_shrink(t, mask, c->N, c->P, shrink, cm->tgt_red.as<double>(), S(stream)));
    }
    return LM_OK;
}

lm_status lm_precond_features(const lm_cache* c, const float* x, const float* M, float* feat, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && x && M && feat, LM_ERR_INVALID_ARG, "lm_precond_features: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    LM_PROF("precond_features", S(stream));
    lm_status st = ensure_gram(cm, S(stream));
    if (st != LM_OK) return st;
    const int64_t N = c->N;
    LM_HIP(cm->coverage.ensure(sizeof(float) * N));
    LM_HIP(cm->feat_red.ensure(sizeof(double) * (12 * lm::feature_parts(N) + 6)));
    LM_HIP(lm::launch_coverage(c->view(), cm->gvgram.as<float>(), cm->coverage.as<float>(), S(stream)));
    LM_HIP(lm::launch_precond_features(M, cm->coverage.as<float>(), x, N, c->P, feat, cm->feat_red.as<double>(),
                                       S(stream)));
    return LM_OK;
}

lm_status lm_apply_JtJ(const lm_cache* c, const float* p, float lambda, const float* M, float* g,
                       double* Jp_sqnorm, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && p && g, LM_ERR_INVALID_ARG, "lm_apply_JtJ: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    lm_status st = apply_JtJ_internal(cm, p, M ? lambda : 0.0f, M, 0.0f, g, nullptr, nullptr, S(stream));
    if (st != LM_OK) return st;
    if (Jp_sqnorm) LM_HIP(lm::reduce_f64(c->jp_part.as<double>(), c->n_tiles, Jp_sqnorm, S(stream)));
    return LM_OK;
}

lm_status lm_apply_J(const lm_cache* c, const float* p, float* u, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && p && u, LM_ERR_INVALID_ARG, "lm_apply_J: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    lm::ApplyBatch B = batch_of(&cm, 1);
    B.a[0].p = p;
    B.a[0].uout = u;
    { LM_PROF("tangent", S(stream)); LM_HIP(lm::launch_tangent(B, S(stream))); }
    { LM_PROF("apply_tile_J", S(stream)); LM_HIP(lm::launch_apply_tile(1, B, S(stream))); }
    return LM_OK;
}

lm_status lm_jp_sqnorm(const lm_cache* c, const float* p, double* out, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && p && out, LM_ERR_INVALID_ARG, "lm_jp_sqnorm: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    lm_cache* cm = const_cast<lm_cache*>(c);
    lm::ApplyBatch B = batch_of(&cm, 1);
    B.a[0].p = p;
    B.a[0].uout = nullptr;   // the J half's per-tile squared norms only
    { LM_PROF("tangent", S(stream)); LM_HIP(lm::launch_tangent(B, S(stream))); }
    { LM_PROF("apply_tile_J", S(stream)); LM_HIP(lm::launch_apply_tile(1, B, S(stream))); }
    LM_HIP(lm::reduce_f64(c->jp_part.as<double>(), c->n_tiles, out, S(stream)));
    return LM_OK;
}

lm_status lm_apply_JT(const lm_cache* c, const float* u, float* g, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && u && g, LM_ERR_INVALID_ARG, "lm_apply_JT: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    return apply_JT_internal(c, u, 1.0f, g, S(stream));
}

// The n_iters iterations of Algorithm 1 for the batch in one cooperative
// launch (persist.hip), after the first product and the initial scalars.
// The launch (counter reset + kernel) is captured into a graph once per
// context, kernel variant and grid, and replayed; where the runtime cannot
// capture a cooperative launch it is issued directly.  Synchronises the
// stream to read the barrier's error flag.
static lm_status pcg_persistent(lm_cache* const* caches, int32_t n_b, const lm::ApplyBatch& B,
                                const float* const* M, const float* const* precond_scale, float* const* delta,
                                float diag_floor, int32_t n_iters, double tol, int32_t tol_mode, hipStream_t s) {
    lm_ctx* cx = lm::g_ctx;
    const int kind = lm::persistent_tile_kind(caches[0]->dtype, caches[0]->thin_k > 0);
    int grid = 0, nt = 0;
    LM_HIP(lm::persistent_grid(caches[0]->deg, kind, &grid, &nt));
    const int n_counters = 2 + LM_PCG_MAX_HISTORY;
    const size_t off_cnt = (sizeof(lm::PersistArgs) + 255) / 256 * 256;
    const size_t off_part = off_cnt + (sizeof(uint32_t) * n_counters + 255) / 256 * 256;
    const size_t need = off_part + sizeof(double) * 3 * lm::kMaxBatch * lm::kPersistMaxGrid;
    if (cx->persist_cap < need) {
        if (cx->persist_dev) {
            LM_HIP(hipStreamSynchronize(s));
            if (cx->persist_al.alloc) cx->persist_al.free(cx->persist_al.user, cx->persist_dev, (void*)cx->persist_stream);
            else LM_HIP(hipFree(cx->persist_dev));
            cx->persist_dev = nullptr;
            cx->persist_cap = 0;
        }
        if (cx->persist_exec) {
            (void)hipGraphExecDestroy(cx->persist_exec);
            cx->persist_exec = nullptr;
        }
        if (cx->al.alloc) {
            cx->persist_dev = cx->al.alloc(cx->al.user, need, (void*)s);
            LM_CHECK(cx->persist_dev, LM_ERR_HIP, "lm_pcg_solve: allocation failed");
        } else {
            LM_HIP(hipMalloc(&cx->persist_dev, need));
        }
        cx->persist_cap = need;
        cx->persist_al = cx->al;
        cx->persist_stream = s;
    }
    char* base = (char*)cx->persist_dev;
    lm::PersistArgs* dev_args = (lm::PersistArgs*)base;
    uint32_t* counters = (uint32_t*)(base + off_cnt);
    // host copy of the arguments, kept in the context until the copy has run
    static thread_local lm::PersistArgs H;
    H = lm::PersistArgs{};
    H.B = B;
    for (int i = 0; i < n_b; ++i) {
        lm_cache* c = caches[i];
        H.B.a[i].stop = nullptr;
        H.B.a[i].pg_part = (double*)(base + off_part);   // non-null: the chain forms p . g
        H.v[i] = lm::PersistSubset{delta[i], c->pcg_r.as<float>(), c->pcg_z.as<float>(), c->pcg_p.as<float>(), M[i],
                                   precond_scale ? precond_scale[i] : nullptr, c->pcg_state.as<lm::PcgState>()};
    }
    H.n = caches[0]->N * (int64_t)caches[0]->P;
    H.n_iters = n_iters;
    H.tol_mode = tol_mode;
    H.tol = tol;
    H.floor_ = diag_floor;
    H.bar = counters;
    H.err = (int32_t*)(counters + 1);
    H.tile_ctr = counters + 2;
    H.part = (double*)(base + off_part);
    LM_HIP(hipMemcpyAsync(dev_args, &H, sizeof(H), hipMemcpyHostToDevice, s));
    {
        LM_PROF("pcg_persistent", s);
        const int key[3] = {caches[0]->deg, kind, grid};
        bool direct = cx->persist_graph == 0;
        if (!direct && (!cx->persist_exec || memcmp(key, cx->persist_key, sizeof(key)) != 0)) {
            if (cx->persist_exec) {
                (void)hipGraphExecDestroy(cx->persist_exec);
                cx->persist_exec = nullptr;
            }
            hipStream_t cs = nullptr;
            LM_HIP(capture_stream(&cs));
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t le = lm::launch_pcg_persistent(dev_args, counters, n_counters, caches[0]->deg, kind,
                                                                grid, cs);
                e = hipStreamEndCapture(cs, &graph);
                if (e == hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&cx->persist_exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                cx->persist_exec = nullptr;
                cx->persist_graph = 0;    // this runtime does not capture cooperative launches
                direct = true;
            } else {
                cx->persist_graph = 1;
                memcpy(cx->persist_key, key, sizeof(key));
            }
        }
        if (direct) LM_HIP(lm::launch_pcg_persistent(dev_args, counters, n_counters, caches[0]->deg, kind, grid, s));
        else LM_HIP(hipGraphLaunch(cx->persist_exec, s));
    }
    int32_t err = 0;
    LM_HIP(hipMemcpyAsync(&err, counters + 1, sizeof(err), hipMemcpyDeviceToHost, s));
    LM_HIP(hipStreamSynchronize(s));
    LM_CHECK(err == 0, LM_ERR_HIP, "lm_pcg_solve: a grid barrier of the persistent kernel timed out");
    return LM_OK;
}

static lm_status pcg_solve_impl(lm_cache* const* caches, int32_t n_b, const float* const* b, const float* const* M,
                                float lambda, float diag_floor, int32_t n_iters, double tol, int32_t tol_mode,
                                const float* const* precond_scale, float* const* delta, lm_pcg_stats* stats,
                                void* stream, bool block) {
    LM_CHECK(caches && b && M && delta && n_b > 0, LM_ERR_INVALID_ARG, "lm_pcg_solve: NULL argument");
    LM_CHECK(n_b <= lm::kMaxBatch, LM_ERR_INVALID_ARG, "lm_pcg_solve: at most 8 subsets per call");
    LM_CHECK(n_iters >= 0 && n_iters < LM_PCG_MAX_HISTORY, LM_ERR_INVALID_ARG, "n_iters out of range");
    LM_CHECK(tol_mode >= LM_TOL_NONE && tol_mode <= LM_TOL_RELATIVE, LM_ERR_INVALID_ARG, "bad tol_mode");
    LM_CHECK(diag_floor >= 0.0f && lambda >= 0.0f, LM_ERR_INVALID_ARG, "lambda and diag_floor must be >= 0");
    hipStream_t s = S(stream);
    for (int i = 0; i < n_b; ++i) {
        const lm_cache* c = caches[i];
        LM_CHECK(c && c->built && b[i] && M[i] && delta[i], LM_ERR_INVALID_ARG, "lm_pcg_solve: bad subset entry");
        LM_CHECK(c->N == caches[0]->N && c->deg == caches[0]->deg && c->dtype == caches[0]->dtype &&
                     (c->thin_k > 0) == (caches[0]->thin_k > 0),
                 LM_ERR_INVALID_ARG, "lm_pcg_solve: subsets must share N, SH degree and cache type");
    }
    const int64_t n = caches[0]->N * (int64_t)caches[0]->P;
    const int64_t nbc = lm::chain_blocks(caches[0]->N);
    // block-Jacobi factors of every subset (before any capture)
    lm::BlockPrecond bjs[lm::kMaxBatch];
    for (int i = 0; i < n_b && block; ++i) {
        lm_status st = ensure_block_precond(caches[i], lambda, diag_floor, s, nullptr);
        if (st != LM_OK) return st;
        bjs[i] = block_precond_of(caches[i]);
    }
    // workspaces and x0 = M^-1 b
    for (int i = 0; i < n_b; ++i) {
        lm_cache* c = caches[i];
        const float* sc = precond_scale ? precond_scale[i] : nullptr;
        const lm::BlockPrecond* bj = block ? &bjs[i] : nullptr;
        LM_HIP(c->pcg_r.ensure(sizeof(float) * n));
        LM_HIP(c->pcg_z.ensure(sizeof(float) * n));
        LM_HIP(c->pcg_p.ensure(sizeof(float) * n));
        LM_HIP(c->pcg_g.ensure(sizeof(float) * n));
        LM_HIP(c->pcg_part.ensure(sizeof(double) * 3 * lm::pcg_partial_count(n)));
        LM_HIP(c->pcg_state.ensure(sizeof(lm::PcgState)));
        LM_HIP(lm::pcg_init(n, b[i], M[i], diag_floor, sc, delta[i], s, bj));
        LM_HIP(hipMemsetAsync(c->pcg_state.p, 0, sizeof(lm::PcgState), s));
    }
    // r0 = b - A x0 for all subsets in one batched product
    lm::ApplyBatch B = batch_of(caches, n_b);
    B.lambda = lambda;
    B.diag_floor = diag_floor;
    for (int i = 0; i < n_b; ++i) {
        B.a[i].p = delta[i];
        B.a[i].M = M[i];
        B.a[i].out = caches[i]->pcg_g.as<float>();
    }
    lm_status e = apply_JtJ_batch(B, s);
    if (e != LM_OK) return e;
    for (int i = 0; i < n_b; ++i) {
        lm_cache* c = caches[i];
        const float* sc = precond_scale ? precond_scale[i] : nullptr;
        LM_HIP(lm::pcg_init_r(n, b[i], c->pcg_g.as<float>(), M[i], diag_floor, sc, c->pcg_r.as<float>(),
                              c->pcg_z.as<float>(), c->pcg_p.as<float>(), c->pcg_part.as<double>(),
                              c->pcg_state.as<lm::PcgState>(), s, block ? &bjs[i] : nullptr));
        B.a[i].p = c->pcg_p.as<float>();
        B.a[i].pg_part = c->pg_part.as<double>();
        B.a[i].stop = &c->pcg_state.as<lm::PcgState>()->stop;
    }
    // one iteration of Algorithm 1 for every subset; the kernels of a subset
    // whose loop has ended return at once
    auto body = [&](hipStream_t q) -> lm_status {
        lm_status st = apply_JtJ_batch(B, q);
        if (st != LM_OK) return st;
        LM_PROF("pcg_vector", q);
        for (int i = 0; i < n_b; ++i) {
            lm_cache* c = caches[i];
            const float* sc = precond_scale ? precond_scale[i] : nullptr;
            lm::PcgState* pst = c->pcg_state.as<lm::PcgState>();
            LM_HIP(lm::pcg_alpha(c->pg_part.as<double>(), nbc, pst, q));
            LM_HIP(lm::pcg_update(n, pst, c->pcg_p.as<float>(), c->pcg_g.as<float>(), M[i], diag_floor, sc, delta[i],
                                  c->pcg_r.as<float>(), c->pcg_z.as<float>(), c->pcg_part.as<double>(), tol, tol_mode,
                                  q, block ? &bjs[i] : nullptr));
        }
        return LM_OK;
    };
    const int mode = lm::g_ctx->pcg_graph;   // 0 eager, 1 graph replay, 2 graph replay for batches, 3 persistent
    const bool use_graph = n_iters >= 2 && (mode == 1 || ((mode == 2 || mode == 3) && n_b > 1));
    if (mode == 3 && !block && n_iters > 0) {
        lm_status ps = pcg_persistent(caches, n_b, B, M, precond_scale, delta, diag_floor, n_iters, tol, tol_mode, s);
        if (ps != LM_OK) return ps;
    } else if (use_graph) {
        // the iteration is captured once (nothing runs while capturing) and
        // replayed on the caller's stream: no host launch work per iteration
        hipStream_t cs = nullptr;
        LM_HIP(capture_stream(&cs));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        LM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        lm::g_ctx->prof.capturing = true;
        lm_status st = body(cs);
        lm::g_ctx->prof.capturing = false;
        hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (st != LM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        LM_HIP(ce);
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            LM_HIP(ie);
        }
        hipError_t le = hipSuccess;
        for (int it = 0; it < n_iters && le == hipSuccess; ++it) {
            LM_PROF("pcg_iteration_graph", s);
            le = hipGraphLaunch(exec, s);
        }
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        LM_HIP(le);
    } else {
        for (int it = 0; it < n_iters; ++it) {
            e = body(s);
            if (e != LM_OK) return e;
        }
    }
    for (int i = 0; i < n_b; ++i) {
        if (!stats) continue;
        lm::PcgState hs;
        LM_HIP(hipMemcpyAsync(&hs, caches[i]->pcg_state.p, sizeof(hs), hipMemcpyDeviceToHost, s));
        LM_HIP(hipStreamSynchronize(s));
        stats[i].iters = hs.iters;
        stats[i].status = hs.status;
        stats[i].b_sqnorm = hs.bb;
        for (int k = 0; k < LM_PCG_MAX_HISTORY; ++k) stats[i].history[k] = k <= hs.iters ? hs.hist[k] : 0.0;
    }
    if (!stats) LM_HIP(hipStreamSynchronize(s));
    return LM_OK;
}

lm_status lm_pcg_solve(lm_cache* const* caches, int32_t n_b, const float* const* b, const float* const* M,
                       float lambda, float diag_floor, int32_t n_iters, double tol, int32_t tol_mode,
                       const float* const* precond_scale, float* const* delta, lm_pcg_stats* stats, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), caches && n_b > 0 && caches[0] ? caches[0]->ctx : nullptr);
    return pcg_solve_impl(caches, n_b, b, M, lambda, diag_floor, n_iters, tol, tol_mode, precond_scale, delta, stats,
                          stream, false);
}

lm_status lm_pcg_solve_block(lm_cache* const* caches, int32_t n_b, const float* const* b, const float* const* M,
                             float lambda, float diag_floor, int32_t n_iters, double tol, int32_t tol_mode,
                             float* const* delta, lm_pcg_stats* stats, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), caches && n_b > 0 && caches[0] ? caches[0]->ctx : nullptr);
    return pcg_solve_impl(caches, n_b, b, M, lambda, diag_floor, n_iters, tol, tol_mode, nullptr, delta, stats,
                          stream, true);
}

lm_status lm_block_precond_apply(lm_cache* c, float lambda, float diag_floor, const float* r, float* z,
                                 int32_t* n_fallback, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && r && z, LM_ERR_INVALID_ARG, "lm_block_precond_apply: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    LM_CHECK(lambda >= 0.0f && diag_floor >= 0.0f, LM_ERR_INVALID_ARG, "lambda and diag_floor must be >= 0");
    lm_status st = ensure_block_precond(c, lambda, diag_floor, S(stream), n_fallback);
    if (st != LM_OK) return st;
    LM_HIP(lm::launch_bj_apply(block_precond_of(c), r, z, S(stream)));
    return n_fallback && *n_fallback > 0 ? LM_WARN_FALLBACK_JACOBI : LM_OK;
}

lm_status lm_autotune_tile(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                           const lm_options* opts, int32_t n_products, void* stream, int32_t* tile_w, int32_t* tile_h,
                           lm_tile_score* scores, int32_t max_scores, int32_t* n_scores) {
    lm::StreamScope lm_stream_scope_(S(stream), opts ? opts->ctx : nullptr);
    const int32_t cache_dtype = opts ? opts->cache_dtype : LM_CACHE_F32;
    LM_CHECK(scene && cams && target && tile_w && tile_h, LM_ERR_INVALID_ARG, "lm_autotune_tile: NULL argument");
    LM_CHECK(n_products >= 0, LM_ERR_INVALID_ARG, "lm_autotune_tile: n_products must be >= 0");
    static const int32_t cand[][2] = {{16, 16}, {32, 8}, {8, 32}, {16, 8}, {8, 16}, {8, 8}};
    const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
    hipStream_t s = S(stream);
    lm_cache* c = nullptr;
    hipEvent_t ev[4] = {};
    for (auto& e : ev) LM_HIP(hipEventCreate(&e));
    const int64_t n = scene->N * (int64_t)(11 + 3 * (scene->sh_degree + 1) * (scene->sh_degree + 1));
    lm_status st = LM_OK;
    // two parameter vectors from the context's allocator
    DevBuf bb, gb;
    hipError_t he = bb.ensure(sizeof(float) * std::max<int64_t>(n, 1));
    if (he == hipSuccess) he = gb.ensure(sizeof(float) * std::max<int64_t>(n, 1));
    float* b = bb.as<float>();
    float* g = gb.as<float>();
    double best = -1.0;
    int found = 0;
    for (int k = 0; k < nc && he == hipSuccess && st == LM_OK; ++k) {
        lm_options o{cand[k][0], cand[k][1], cache_dtype, 0, nullptr, lm::g_ctx, opts ? opts->thin_window : 0, 0};
        // an untimed build first: buffer growth (device allocation) is not
        // part of the shape's cost
        st = lm_build_cache(scene, cams, V, target, &o, stream, &c, b, nullptr);
        if (st != LM_OK) break;
        he = hipEventRecord(ev[0], s);
        if (he != hipSuccess) break;
        st = lm_build_cache(scene, cams, V, target, &o, stream, &c, b, nullptr);
        if (st != LM_OK) break;
        he = hipEventRecord(ev[1], s);
        // one untimed product, then two timed ones, along b = -J^T F
        if (he == hipSuccess) st = apply_JtJ_internal(c, b, 0.0f, nullptr, 0.0f, g, nullptr, nullptr, s);
        if (st != LM_OK) break;
        he = hipEventRecord(ev[2], s);
        for (int r = 0; r < 2 && st == LM_OK && he == hipSuccess; ++r)
            st = apply_JtJ_internal(c, b, 0.0f, nullptr, 0.0f, g, nullptr, nullptr, s);
        if (st != LM_OK) break;
        if (he == hipSuccess) he = hipEventRecord(ev[3], s);
        if (he == hipSuccess) he = hipEventSynchronize(ev[3]);
        float build_ms = 0.0f, apply_ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&build_ms, ev[0], ev[1]);
        if (he == hipSuccess) he = hipEventElapsedTime(&apply_ms, ev[2], ev[3]);
        if (he != hipSuccess) break;
        apply_ms *= 0.5f;
        const double score = build_ms + (double)n_products * apply_ms;
        if (scores && found < max_scores) scores[found] = lm_tile_score{cand[k][0], cand[k][1], build_ms, apply_ms};
        ++found;
        if (best < 0.0 || score < best) {
            best = score;
            *tile_w = cand[k][0];
            *tile_h = cand[k][1];
        }
    }
    if (n_scores) *n_scores = std::min(found, max_scores);
    (void)hipStreamSynchronize(s);
    if (c) lm_cache_destroy(c);
    bb.release();
    gb.release();
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != LM_OK) return st;
    LM_HIP(he);
    LM_CHECK(best >= 0.0, LM_ERR_INVALID_ARG, "lm_autotune_tile: no candidate could be measured");
    return LM_OK;
}

lm_status lm_set_allocator(const lm_allocator* a) {
    LM_CHECK(!a || (a->alloc && a->free), LM_ERR_INVALID_ARG, "lm_set_allocator: alloc and free are both required");
    lm::g_default_ctx.al = a ? *a : lm_allocator{};
    return LM_OK;
}

lm_status lm_pcg_use_graph(lm_ctx* ctx, int32_t mode) {
    LM_CHECK(mode >= 0 && mode <= 3, LM_ERR_INVALID_ARG, "lm_pcg_use_graph: mode must be 0, 1, 2 or 3");
    (ctx ? ctx : &lm::g_default_ctx)->pcg_graph = mode;
    return LM_OK;
}

lm_status lm_profile_enable(lm_ctx* ctx, int32_t on) {
    (ctx ? ctx : &lm::g_default_ctx)->prof.enabled = on != 0;
    return LM_OK;
}

int32_t lm_profile_read(lm_ctx* ctx, lm_profile_entry* out, int32_t max_entries) {
    lm::prof::State& P = (ctx ? ctx : &lm::g_default_ctx)->prof;
    struct Agg {
        std::string name;
        int32_t n = 0;
        double ms = 0.0;
    };
    std::vector<Agg> agg;
    for (const lm::prof::Rec& r : P.recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.0f;
        auto it = std::find_if(agg.begin(), agg.end(), [&](const Agg& x) { return x.name == r.name; });
        if (it == agg.end()) {
            agg.push_back({r.name, 0, 0.0});
            it = agg.end() - 1;
        }
        it->n += 1;
        it->ms += ms;
    }
    P.recs.clear();
    P.used = 0;
    std::sort(agg.begin(), agg.end(), [](const Agg& a, const Agg& b) { return a.name < b.name; });
    int32_t k = 0;
    for (const Agg& a : agg) {
        if (!out || k >= max_entries) break;
        memset(&out[k], 0, sizeof(out[k]));
        strncpy(out[k].name, a.name.c_str(), sizeof(out[k].name) - 1);
        out[k].launches = a.n;
        out[k].total_ms = a.ms;
        ++k;
    }
    return k;
}

lm_status lm_combine_subsets(int32_t n_b, const float* const* delta, const float* const* M, int64_t n, float* out,
                             void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream));
    LM_CHECK(delta && M && out && n_b > 0 && n_b <= 16 && n >= 0, LM_ERR_INVALID_ARG,
             "lm_combine_subsets: bad arguments (1 <= n_b <= 16)");
    for (int i = 0; i < n_b; ++i) LM_CHECK(delta[i] && M[i], LM_ERR_INVALID_ARG, "lm_combine_subsets: NULL entry");
    if (n == 0) return LM_OK;
    { LM_PROF("combine", S(stream)); LM_HIP(lm::launch_combine(n_b, delta, M, n, out, S(stream))); }
    return LM_OK;
}

lm_status lm_mlp_forward(const float* w, const float* feat, int64_t n, int32_t p_out, float* s, float* scale,
                         uint32_t* n_fallback, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream));
    LM_CHECK(w && (n == 0 || feat) && n >= 0, LM_ERR_INVALID_ARG, "lm_mlp_forward: bad argument");
    LM_CHECK(p_out >= 1 && p_out <= LM_MLP_MAX_OUT, LM_ERR_INVALID_ARG, "lm_mlp_forward: p_out must be 1..64");
    LM_CHECK(n < ((int64_t)1 << 40), LM_ERR_CAPACITY, "lm_mlp_forward: n too large");
    if (n_fallback) LM_HIP(hipMemsetAsync(n_fallback, 0, sizeof(uint32_t), S(stream)));
    {
        LM_PROF("mlp_forward", S(stream));
        LM_HIP(lm::launch_mlp_forward(w, feat, n, p_out, s, scale, n_fallback, S(stream)));
    }
    if (n_fallback) {
        // the count decides the warning: read it back
        uint32_t h = 0;
        LM_HIP(hipMemcpyAsync(&h, n_fallback, sizeof(h), hipMemcpyDeviceToHost, S(stream)));
        LM_HIP(hipStreamSynchronize(S(stream)));
        if (h > 0) return LM_WARN_FALLBACK_JACOBI;
    }
    return LM_OK;
}

size_t lm_mlp_workspace_bytes(void) {
    const size_t parts = (size_t)lm::mlp_grad_parts();
    return parts * lm::kMlpParams * sizeof(float) + parts * 2 * sizeof(double);
}

lm_status lm_mlp_train_step(float* w, float* adam_m, float* adam_v, int32_t step, float lr, const float* feat,
                            const float* target, const float* mask, int64_t n, int32_t p_out, float* grad,
                            double* loss, void* workspace, size_t workspace_bytes, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream));
    LM_CHECK(w && (n == 0 || (feat && target && mask)) && n >= 0, LM_ERR_INVALID_ARG,
             "lm_mlp_train_step: bad argument");
    LM_CHECK(p_out >= 1 && p_out <= LM_MLP_MAX_OUT, LM_ERR_INVALID_ARG, "lm_mlp_train_step: p_out must be 1..64");
    LM_CHECK(!(lr > 0.0f) || (adam_m && adam_v && step >= 1), LM_ERR_INVALID_ARG,
             "lm_mlp_train_step: lr > 0 needs adam_m, adam_v and step >= 1");
    LM_CHECK(lr >= 0.0f, LM_ERR_INVALID_ARG, "lm_mlp_train_step: lr must be >= 0");
    LM_CHECK(workspace && workspace_bytes >= lm_mlp_workspace_bytes(), LM_ERR_INVALID_ARG,
             "lm_mlp_train_step: workspace smaller than lm_mlp_workspace_bytes()");
    LM_CHECK(n < ((int64_t)1 << 40), LM_ERR_CAPACITY, "lm_mlp_train_step: n too large");
    const size_t parts = (size_t)lm::mlp_grad_parts();
    float* gpart = static_cast<float*>(workspace);
    double* lpart = reinterpret_cast<double*>(gpart + parts * lm::kMlpParams);
    LM_PROF("mlp_train_step", S(stream));
    LM_HIP(lm::launch_mlp_grad_step(w, adam_m, adam_v, step, lr, feat, target, mask, n, p_out, grad, loss, gpart,
                                    lpart, S(stream)));
    return LM_OK;
}

lm_status lm_render(const lm_scene* scene, const lm_camera* cams, int32_t V, const lm_options* opts, float* image,
                    void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), opts ? opts->ctx : nullptr);
    LM_CHECK(image, LM_ERR_INVALID_ARG, "lm_render: image is NULL");
    lm_cache* c = new (std::nothrow) lm_cache();
    LM_CHECK(c, LM_ERR_HIP, "out of host memory");
    hipStream_t s = S(stream);
    lm_status st = build_forward(c, scene, cams, V, nullptr, opts, s, false);
    if (st == LM_OK) {
        hipError_t e = hipMemcpyAsync(image, c->resid.p, sizeof(float) * 3 * c->n_pix, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            lm::set_error(std::string("lm_render: ") + hipGetErrorString(e));
            st = LM_ERR_HIP;
        }
    }
    (void)hipStreamSynchronize(s);
    c->release_all();
    delete c;
    return st;
}

lm_status lm_residual_sqnorm(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                             const lm_options* opts, void* stream, lm_cache** workspace, double* F_sqnorm) {
    lm::StreamScope lm_stream_scope_(S(stream), opts ? opts->ctx : nullptr);
    LM_CHECK(workspace && target && F_sqnorm, LM_ERR_INVALID_ARG, "lm_residual_sqnorm: NULL argument");
    lm_cache* c = *workspace;
    bool created = false;
    if (!c) {
        c = new (std::nothrow) lm_cache();
        LM_CHECK(c, LM_ERR_HIP, "out of host memory");
        created = true;
    }
    bind_ctx(c);
    hipStream_t s = S(stream);
    lm_status st = build_forward(c, scene, cams, V, target, opts, s, false);
    if (st == LM_OK) {
        hipError_t e = lm::reduce_f64(c->fsq_part.as<double>(), c->n_tiles, F_sqnorm, s);
        if (e != hipSuccess) {
            lm::set_error(std::string("lm_residual_sqnorm: ") + hipGetErrorString(e));
            st = LM_ERR_HIP;
        }
    }
    c->built = false;
    if (st != LM_OK && created) {
        free_handle(c);
        return st;
    }
    *workspace = c;
    return st;
}

lm_status lm_cache_view_sqnorm(const lm_cache* c, double* per_view, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && per_view, LM_ERR_INVALID_ARG, "lm_cache_view_sqnorm: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    LM_HIP(lm::view_sum_f64(c->cams.as<lm::CamDev>(), c->V, c->fsq_part.as<double>(), per_view, S(stream)));
    return LM_OK;
}

lm_status lm_objective_terms(const float* image, const float* target, const lm_camera* cams, int32_t V,
                             const lm_objective* obj, float* w, float* e, double* E, void* stream,
                             lm_cache** workspace) {
    lm::StreamScope lm_stream_scope_(S(stream), workspace && *workspace ? (*workspace)->ctx : nullptr);
    LM_CHECK(image && target && cams && E && workspace, LM_ERR_INVALID_ARG, "lm_objective_terms: NULL argument");
    LM_CHECK(V > 0 && V <= lm::kMaxViews, LM_ERR_INVALID_ARG, "lm_objective_terms: bad view count");
    lm_status st = objective_check(obj);
    if (st != LM_OK) return st;
    std::vector<int> Ws(V), Hs(V);
    for (int v = 0; v < V; ++v) {
        LM_CHECK(cams[v].W > 0 && cams[v].H > 0, LM_ERR_INVALID_ARG, "camera with empty image");
        Ws[v] = cams[v].W;
        Hs[v] = cams[v].H;
    }
    lm_cache* c = *workspace;
    bool created = false;
    if (!c) {
        c = new (std::nothrow) lm_cache();
        LM_CHECK(c, LM_ERR_HIP, "out of host memory");
        created = true;
    }
    bind_ctx(c);
    st = run_objective(c, image, target, false, Ws, Hs, obj, w, e, E, nullptr, nullptr, S(stream));
    if (st != LM_OK && created) {
        free_handle(c);
        return st;
    }
    *workspace = c;
    return st;
}

lm_status lm_set_residual_weights(lm_cache* c, const float* w, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c, LM_ERR_INVALID_ARG, "lm_set_residual_weights: NULL cache");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    c->gram_valid = false;
    c->bj_valid = false;
    if (!w) {
        c->weighted = false;
        return LM_OK;
    }
    LM_HIP(c->wres.ensure(sizeof(float) * 3 * c->n_pix));
    LM_HIP(hipMemcpyAsync(c->wres.p, w, sizeof(float) * 3 * c->n_pix, hipMemcpyDeviceToDevice, S(stream)));
    c->weighted = true;
    return LM_OK;
}

lm_status lm_cache_objective(lm_cache* c, const float* target, const lm_objective* obj, float* b, double* E,
                             void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && target, LM_ERR_INVALID_ARG, "lm_cache_objective: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    LM_CHECK(!c->compact, LM_ERR_NOT_BUILT,
             "lm_cache_objective: the residual image was released (LM_BUILD_COMPACT build)");
    lm_status st = objective_check(obj);
    if (st != LM_OK) return st;
    hipStream_t s = S(stream);
    c->gram_valid = false;
    c->bj_valid = false;
    if (obj->kind == LM_OBJ_L2) {
        c->weighted = false;
        if (E) LM_HIP(lm::view_sum_f64(c->cams.as<lm::CamDev>(), c->V, c->fsq_part.as<double>(), E, s));
        if (b) return apply_JT_internal(c, c->resid.as<float>(), -1.0f, b, s);
        return LM_OK;
    }
    LM_HIP(c->wres.ensure(sizeof(float) * 3 * c->n_pix));
    LM_HIP(c->obj_e.ensure(sizeof(float) * 3 * c->n_pix));
    std::vector<int> Ws(c->V), Hs(c->V);
    for (int v = 0; v < c->V; ++v) {
        Ws[v] = c->cams_h[v].W;
        Hs[v] = c->cams_h[v].H;
    }
    {
        LM_PROF("objective", s);
        st = run_objective(c, c->resid.as<float>(), target, true, Ws, Hs, obj, c->wres.as<float>(),
                           c->obj_e.as<float>(), nullptr, c->cams.as<lm::CamDev>(), E, s);
    }
    if (st != LM_OK) return st;
    c->weighted = true;
    if (b) return apply_JT_internal(c, c->obj_e.as<float>(), -1.0f, b, s);
    return LM_OK;
}

lm_status lm_objective_value(const lm_scene* scene, const lm_camera* cams, int32_t V, const float* target,
                             const lm_options* opts, const lm_objective* obj, void* stream, lm_cache** workspace,
                             double* E) {
    lm::StreamScope lm_stream_scope_(S(stream), opts ? opts->ctx : nullptr);
    LM_CHECK(workspace && target && E, LM_ERR_INVALID_ARG, "lm_objective_value: NULL argument");
    lm_status st = objective_check(obj);
    if (st != LM_OK) return st;
    lm_cache* c = *workspace;
    bool created = false;
    if (!c) {
        c = new (std::nothrow) lm_cache();
        LM_CHECK(c, LM_ERR_HIP, "out of host memory");
        created = true;
    }
    bind_ctx(c);
    hipStream_t s = S(stream);
    st = build_forward(c, scene, cams, V, target, opts, s, false);
    if (st == LM_OK) {
        if (obj->kind == LM_OBJ_L2) {
            hipError_t e = lm::reduce_f64(c->fsq_part.as<double>(), c->n_tiles, E, s);
            if (e != hipSuccess) {
                lm::set_error(std::string("lm_objective_value: ") + hipGetErrorString(e));
                st = LM_ERR_HIP;
            }
        } else {
            std::vector<int> Ws(V), Hs(V);
            for (int v = 0; v < V; ++v) {
                Ws[v] = cams[v].W;
                Hs[v] = cams[v].H;
            }
            st = run_objective(c, c->resid.as<float>(), target, true, Ws, Hs, obj, nullptr, nullptr, E, nullptr,
                               nullptr, s);
        }
    }
    c->built = false;
    if (st != LM_OK && created) {
        free_handle(c);
        return st;
    }
    *workspace = c;
    return st;
}

int64_t lm_cache_export_size(const lm_cache* c, int32_t what) {
    if (!c || !c->built) return -1;
    switch (what) {
        case LM_EXPORT_RECORDS_F32: return 4 * 4 * c->N * (int64_t)c->V;
        case LM_EXPORT_SORTED_VALUES: return 4 * c->n_keys;
        case LM_EXPORT_TILE_RANGES: return 8 * (c->n_tiles + 1);
        case LM_EXPORT_IMAGE: return 4 * 3 * c->n_pix;
        case LM_EXPORT_NCONTRIB: return 4 * c->n_pix;
        case LM_EXPORT_PAIR_T: return 4 * c->n_pairs;
        case LM_EXPORT_PAIR_D: return 4 * 3 * c->n_pairs;
        case LM_EXPORT_PAIR_PIX: return 4 * c->n_pairs;
        case LM_EXPORT_PAIR_GAUSS: return 4 * c->n_pairs;
        case LM_EXPORT_RESIDUAL: return 4 * 3 * c->n_pix;
        case LM_EXPORT_PAIR_FLAGS: return 4 * c->n_pairs;
        case LM_EXPORT_TILE_SEGMENTS: return 8 * (c->n_tiles + 1);
        default: return -1;
    }
}

}  // extern "C"

namespace {

float decode_word(const uint8_t* base, int dtype, int64_t i, uint32_t* flags) {
    if (dtype == LM_CACHE_F32) {
        uint32_t w;
        memcpy(&w, base + 4 * i, 4);
        if (flags) *flags = ((w >> 31) & 1u) | (((w >> 30) & 1u) << 1);
        if (flags) w &= 0x3FFFFFFFu;
        float f;
        memcpy(&f, &w, 4);
        return f;
    }
    uint16_t h;
    memcpy(&h, base + 2 * i, 2);
    if (flags) {
        *flags = ((h >> 15) & 1u) | (((h >> 14) & 1u) << 1);
        h &= 0x3FFF;
    }
    if (dtype == LM_CACHE_BF16) {
        uint32_t w = (uint32_t)h << 16;
        float f;
        memcpy(&f, &w, 4);
        return f;
    }
    // binary16 -> float
    const uint32_t sign = (h >> 15) & 1u, ex = (h >> 10) & 0x1Fu, man = h & 0x3FFu;
    float mag;
    if (ex == 0) mag = ldexpf((float)man, -24);
    else if (ex == 31) mag = man ? NAN : INFINITY;
    else mag = ldexpf((float)(man | 0x400u), (int)ex - 25);
    return sign ? -mag : mag;
}

template <class T>
hipError_t fetch(std::vector<T>& out, const void* dev, int64_t n, hipStream_t s) {
    out.resize((size_t)std::max<int64_t>(n, 0));
    if (n <= 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(out.data(), dev, sizeof(T) * n, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Pair slots holding a pair, in slot order (the zero slots pad each segment
// to a multiple of 8; a stored T is >= 1e-4, so its word is never zero).
hipError_t live_slots(const lm_cache* c, std::vector<int64_t>& live, hipStream_t s) {
    const size_t wb = lm::dtype_bytes(c->dtype);
    std::vector<uint8_t> raw;
    hipError_t e = fetch(raw, c->pT.p, (int64_t)wb * c->n_slots, s);
    if (e != hipSuccess) return e;
    live.clear();
    live.reserve((size_t)c->n_pairs);
    for (int64_t i = 0; i < c->n_slots; ++i) {
        bool nz = false;
        for (size_t b = 0; b < wb; ++b) nz |= raw[(size_t)i * wb + b] != 0;
        if (nz) live.push_back(i);
    }
    return hipSuccess;
}

}  // namespace

extern "C" lm_status lm_cache_export(const lm_cache* c, int32_t what, void* host_dst, int64_t bytes, void* stream) {
    lm::StreamScope lm_stream_scope_(S(stream), c ? c->ctx : nullptr);
    LM_CHECK(c && host_dst, LM_ERR_INVALID_ARG, "lm_cache_export: NULL argument");
    LM_CHECK(c->built, LM_ERR_NOT_BUILT, "cache not built");
    const int64_t need = lm_cache_export_size(c, what);
    LM_CHECK(need >= 0, LM_ERR_INVALID_ARG, "lm_cache_export: unknown array");
    LM_CHECK(bytes == need, LM_ERR_INVALID_ARG, "lm_cache_export: size mismatch");
    hipStream_t s = S(stream);
    const int64_t R = c->N * (int64_t)c->V;
    const bool build_only = what == LM_EXPORT_RECORDS_F32 || what == LM_EXPORT_SORTED_VALUES ||
                            what == LM_EXPORT_TILE_RANGES || what == LM_EXPORT_IMAGE ||
                            what == LM_EXPORT_NCONTRIB || what == LM_EXPORT_RESIDUAL;
    LM_CHECK(!(c->compact && build_only), LM_ERR_INVALID_ARG,
             "lm_cache_export: the build buffers of this cache were released (LM_BUILD_COMPACT)");
    const bool pair_array = what == LM_EXPORT_PAIR_T || what == LM_EXPORT_PAIR_D || what == LM_EXPORT_PAIR_PIX ||
                            what == LM_EXPORT_PAIR_GAUSS || what == LM_EXPORT_PAIR_FLAGS;
    LM_CHECK(!(c->thin_k && pair_array), LM_ERR_UNSUPPORTED,
             "lm_cache_export: a thinned cache stores no per-pair values");
    switch (what) {
        case LM_EXPORT_RECORDS_F32: {
            std::vector<float> rf;
            std::vector<int32_t> rd;
            LM_HIP(fetch(rf, c->recf.p, 3 * R, s));
            LM_HIP(fetch(rd, c->rad.p, R, s));
            float* o = (float*)host_dst;
            for (int64_t r = 0; r < R; ++r) {
                o[4 * r] = rf[r];
                o[4 * r + 1] = rf[R + r];
                o[4 * r + 2] = rf[2 * R + r];
                o[4 * r + 3] = (float)rd[r];
            }
            return LM_OK;
        }
        case LM_EXPORT_SORTED_VALUES:
            if (c->n_keys) {
                LM_HIP(hipMemcpyAsync(host_dst, c->sorted_vals(), bytes, hipMemcpyDeviceToHost, s));
                LM_HIP(hipStreamSynchronize(s));
            }
            return LM_OK;
        case LM_EXPORT_TILE_RANGES:
            LM_HIP(hipMemcpyAsync(host_dst, c->tile_start.p, bytes, hipMemcpyDeviceToHost, s));
            LM_HIP(hipStreamSynchronize(s));
            return LM_OK;
        case LM_EXPORT_TILE_SEGMENTS:
            LM_HIP(hipMemcpyAsync(host_dst, c->tile_seg_off.p, bytes, hipMemcpyDeviceToHost, s));
            LM_HIP(hipStreamSynchronize(s));
            return LM_OK;
        case LM_EXPORT_IMAGE: {
            // rendered colour = residual + target is not stored; the float64
            // colour per pixel is, in [3][n_pix] order
            std::vector<double> pc;
            LM_HIP(fetch(pc, c->pixC.p, 3 * c->n_pix, s));
            float* o = (float*)host_dst;
            for (int v = 0; v < c->V; ++v) {
                const lm::CamDev& cam = c->cams_h[v];
                const int64_t HW = (int64_t)cam.W * cam.H;
                for (int ch = 0; ch < 3; ++ch)
                    for (int64_t i = 0; i < HW; ++i)
                        o[3 * cam.pix_base + ch * HW + i] = (float)pc[ch * c->n_pix + cam.pix_base + i];
            }
            return LM_OK;
        }
        case LM_EXPORT_NCONTRIB:
            LM_HIP(hipMemcpyAsync(host_dst, c->ncontrib.p, bytes, hipMemcpyDeviceToHost, s));
            LM_HIP(hipStreamSynchronize(s));
            return LM_OK;
        case LM_EXPORT_RESIDUAL:
            LM_HIP(hipMemcpyAsync(host_dst, c->resid.p, bytes, hipMemcpyDeviceToHost, s));
            LM_HIP(hipStreamSynchronize(s));
            return LM_OK;
        case LM_EXPORT_PAIR_T:
        case LM_EXPORT_PAIR_FLAGS: {
            const size_t wb = lm::dtype_bytes(c->dtype);
            std::vector<uint8_t> raw;
            std::vector<int64_t> live;
            LM_HIP(live_slots(c, live, s));
            LM_HIP(fetch(raw, c->pT.p, (int64_t)wb * c->n_slots, s));
            for (size_t i = 0; i < live.size(); ++i) {
                uint32_t fl = 0;
                const float v = decode_word(raw.data(), c->dtype, live[i], &fl);
                if (what == LM_EXPORT_PAIR_T) ((float*)host_dst)[i] = v;
                else ((int32_t*)host_dst)[i] = (int32_t)fl;
            }
            return LM_OK;
        }
        case LM_EXPORT_PAIR_D: {
            const size_t wb = lm::dtype_bytes(c->dtype);
            std::vector<uint8_t> raw;
            std::vector<int64_t> live;
            LM_HIP(live_slots(c, live, s));
            LM_HIP(fetch(raw, c->pD.p, (int64_t)wb * 3 * c->pair_stride, s));
            for (int ch = 0; ch < 3; ++ch)
                for (size_t i = 0; i < live.size(); ++i)
                    ((float*)host_dst)[ch * c->n_pairs + (int64_t)i] =
                        decode_word(raw.data(), c->dtype, ch * c->pair_stride + live[i], nullptr);
            return LM_OK;
        }
        case LM_EXPORT_PAIR_PIX:
        case LM_EXPORT_PAIR_GAUSS: {
            // every live slot in slot order: its tile from the tile offsets,
            // its segment from the run table
            std::vector<uint64_t> tpo;
            std::vector<uint32_t> rseg, sgv, gvrec;
            std::vector<uint8_t> pix;
            LM_HIP(fetch(tpo, c->tile_pair_off.p, c->n_tiles + 1, s));
            LM_HIP(fetch(rseg, c->run_seg.p, c->n_slots / 8, s));
            LM_HIP(fetch(sgv, c->seg_gv.p, c->n_seg, s));
            LM_HIP(fetch(gvrec, c->gv_rec.p, c->n_gv, s));
            LM_HIP(fetch(pix, c->ppix.p, c->n_slots, s));
            std::vector<int64_t> live;
            LM_HIP(live_slots(c, live, s));
            std::vector<int32_t> tview;
            for (int v = 0; v < c->V; ++v) {
                const lm::CamDev& cam = c->cams_h[v];
                tview.insert(tview.end(), (size_t)cam.TX * cam.TY, v);
            }
            int32_t* o = (int32_t*)host_dst;
            int64_t t = 0;
            for (size_t k = 0; k < live.size(); ++k) {
                const int64_t q = live[k];
                while (t + 1 < c->n_tiles && (int64_t)tpo[t + 1] <= q) ++t;
                if (what == LM_EXPORT_PAIR_GAUSS) {
                    o[k] = (int32_t)(gvrec[sgv[rseg[q / 8]]] % (uint64_t)c->N);
                } else {
                    const lm::CamDev& cam = c->cams_h[tview[t]];
                    const int64_t lt = t - cam.tile_base;
                    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
                    const int pl = pix[q];
                    const int px = tx * c->TW + pl % c->TW, py = ty * c->TH + pl / c->TW;
                    o[k] = (int32_t)(cam.pix_base + (int64_t)py * cam.W + px);
                }
            }
            return LM_OK;
        }
        default:
            break;
    }
    lm::set_error("lm_cache_export: unknown array");
    return LM_ERR_INVALID_ARG;
}
