// Forward rasterisation and gradient-cache construction (Algorithm 1,
// buildCache; section 3.3 "Cache-driven parallelization").
//
// One workgroup per tile, one thread per pixel.  Each batch of up to 256
// entries of the tile's depth-sorted list is staged in LDS (float64 splat
// data) and every pixel walks it front to back (eq. alpha-blending):
//     power = -0.5 (A dx^2 + C dy^2) - B dx dy   (skip if > 0)
//     alpha = min(0.99, o exp(power))            (skip if < 1/255)
//     stop (without this splat) if T (1 - alpha) < 1e-4
//     C += c alpha T,  T *= 1 - alpha.
// Blending state and every decision are float64, so the contributing set is
// the float64 one.
//
// Two passes walk identically:
//   count: per entry, contributing pixels per wave (packed 4 x u8); per pixel
//          the rendered colour (float64), residual and contributor count;
//          per tile the number of pairs (per pixel block, padded) and of
//          active splats (segments).
//   fill:  writes the cache in its final layout.  A tile's pixels form up
//          to four blocks of 64 (the pixels of one wave: an 8x8 square when
//          the tile is at least 8 pixels each way, else 64 consecutive
//          pixels).  Per tile, block after block; within a block, the active
//          splats in depth order, each with its pairs in that block (a
//          piece) in lane order, rotated within each run of 8 by the
//          segment index: T (with head/clamp flag bits), dC/dalpha (3
//          planes), pixel byte.  Every piece starts on a multiple of 8
//          pairs (zero padding), so each aligned run of 8 pairs belongs to
//          one segment (the splat's pieces in the tile) and one block; the
//          run -> segment table names it.  No piece crosses a multiple of
//          kWindow pairs from its block's start (it moves to the next one;
//          the gap is zero-filled and its runs are named by the piece's
//          segment): the product and Gram passes give each wave kWindow
//          pairs at a time, so every piece is summed by one wave and each
//          segment gets one addition per block, in block order
//          (deterministic sums).  A block's pairs are complete for its 64
//          pixels, so the product pass can finish u = J p of a block and
//          run J^T on the same pairs while they are on chip.
//          Per segment: the splat data and the (Gaussian, view) links.
//   thin fill (a thinned cache, thin_k = K > 0): per block the active
//          splats in depth order as pieces (segment, 64-bit mask of the
//          block's pixels it contributes to, mask of those where its alpha
//          is clamped); per pixel, for its contributors 0, K, 2K, ...: the
//          transmittance in front of it and the colour still to be blended
//          from it on (float32 x 4); per segment also the splat's colour.
// dC_ch/dalpha = T c_ch - S_ch/(1 - alpha) with S_ch the colour blended by
// later splats, S_ch = C_ch(final) - (colour blended up to and including
// this splat), all in float64.
#include "lm_internal.h"

namespace lm {
namespace {

constexpr int NW = kBlock / kWave;



__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }
__device__ __forceinline__ uint32_t pad8(uint32_t n) { return (n + 7u) & ~7u; }
// Placement of a block's pieces in depth order: a piece of len padded pairs
// (len <= 64 <= kWindow) starts where the previous one ends, moved to the
// next window when it would cross one.  64 consecutive pieces at once (one
// wave; lane j holds piece j's padded length, 0 for none): an exclusive scan
// of the lengths puts each piece at the end of the one before; then, lane
// by lane in order, the first piece that would cross a window moves to the
// next one and every later piece moves with it.  gap: the end of the
// previous piece; off: this piece's start; returns the block's new end (in
// every lane).  With windows false no piece moves.
__device__ __forceinline__ uint32_t place_wave(uint32_t e, uint32_t len, bool windows, uint32_t& gap,
                                               uint32_t& off) {
    const int lane = __lane_id();
    uint32_t inc = len;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    const uint32_t ex = inc - len;
    uint32_t prev = 0, own = 0;       // moves of the earlier pieces, of this one
    if (windows) {
        int fixed = -1;               // lanes up to here are placed
        for (;;) {
            const uint32_t st = e + ex + prev;
            const bool cross = lane > fixed && len > 0 && (st & (kWindow - 1)) + len > kWindow;
            const uint64_t m = __ballot(cross);
            if (m == 0ull) break;
            const int f = __ffsll((unsigned long long)m) - 1;
            const uint32_t sf = (uint32_t)__builtin_amdgcn_readlane((int)st, f);
            const uint32_t add = kWindow - (sf & (kWindow - 1));
            if (lane == f) own = add;
            if (lane > f) prev += add;
            fixed = f;
        }
    }
    gap = e + ex + prev;
    off = gap + own;
    return (uint32_t)__builtin_amdgcn_readlane((int)(off + len), kWave - 1);
}

template <bool FILL, int DT, bool THIN>
__global__ void __launch_bounds__(kBlock) k_raster(RasterArgs a) {
    using S = Store<DT>;
    __shared__ double s_rec[10][kBlock];
    __shared__ uint32_t s_g[kBlock];
    __shared__ uint8_t s_wc[kBlock][NW];       // count pass: contributing pixels per wave
    __shared__ uint32_t s_eoff[kBlock][NW];    // fill pass: tile offset of each entry's piece per block
    __shared__ uint32_t s_egap[kBlock][NW];    // fill pass: tile offset of the gap before it (its start if none)
    __shared__ uint32_t s_cnt[kBlock];         // fill pass: the batch's per-entry counts
    __shared__ uint32_t s_eseg[kBlock];        // fill pass: segment of each active entry
    __shared__ uint16_t s_act[kBlock];         // fill pass: the batch's active entries in depth order
    __shared__ uint32_t s_run[3];              // running -, segments, real pairs
    __shared__ uint32_t s_blk[NW];             // running padded pairs per block (count); block starts (fill)
    __shared__ double s_red[kBlock / kWave];
    __shared__ uint32_t s_scan4[NW][4];

    const int64_t t = blockIdx.x;
    const int v = a.tile_view[t];
    const CamDev& cam = a.cams[v];
    const int64_t lt = t - cam.tile_base;
    const int tx = (int)(lt % cam.TX), ty = (int)(lt / cam.TX);
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid / kWave;
    // each wave takes an 8x8 block of the tile (when the tile is at least
    // 8 pixels each way): compact waves share splats and saturate together
    int lx, ly;
    if (a.TW >= 8 && a.TH >= 8) {
        const int blk = tid >> 6, bpr = a.TW >> 3;
        lx = ((blk % bpr) << 3) + (tid & 7);
        ly = ((blk / bpr) << 3) + ((tid >> 3) & 7);
    } else {
        lx = tid % a.TW;
        ly = tid / a.TW;
    }
    const int px = tx * a.TW + lx, py = ty * a.TH + ly;
    const bool valid = tid < a.TW * a.TH && px < cam.W && py < cam.H;
    const double pxc = px + 0.5, pyc = py + 0.5;
    const int64_t pg = cam.pix_base + (int64_t)py * cam.W + px;   // global pixel index
    const int64_t HW = (int64_t)cam.W * cam.H;
    const int64_t R = a.N * (int64_t)a.V;

    double T = 1.0, acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    double Ch0 = 0.0, Ch1 = 0.0, Ch2 = 0.0;
    int cnt = 0;
    bool done = !valid;
    // tile-relative key at which the pixel saturates (the count pass finds it
    // and a build stores it; the fill pass reads it): no later key reaches it
    uint32_t stop = (FILL && valid) ? a.pix_stop[pg] : 0xFFFFFFFFu;
    if (FILL && valid) {
        Ch0 = a.pixC[pg];
        Ch1 = a.pixC[a.n_pix + pg];
        Ch2 = a.pixC[2 * a.n_pix + pg];
    }
    if (tid < 3) s_run[tid] = 0;
    if (tid < NW) s_blk[tid] = 0;
    int64_t pair_base = 0, seg_base = 0, pair_end = 0, seg_end = 0;
    uint32_t blk_end = 0;       // end of this wave's block in the tile (fill)
    if (FILL) {
        pair_base = a.tile_pair_off[t];
        seg_base = a.tile_seg_off[t];
        pair_end = a.tile_pair_off[t + 1];
        seg_end = a.tile_seg_off[t + 1];
        for (int w = 0; w <= wid; ++w) blk_end += a.tile_blk[t * kTileBlocks + w];
    }
    __shared__ uint32_t s_bbase[NW];           // fill: first slot of each block in the tile
    if (FILL && tid == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < NW; ++w) {
            s_bbase[w] = acc;
            acc += a.tile_blk[t * kTileBlocks + w];
        }
    }
    const int64_t ks = a.tile_start[t], ke = a.tile_start[t + 1];
    const double lmargin = 1e-9;
    // thin fill: this pixel's checkpoints (one per K contributors) in the
    // tile's checkpoint range, pixels in thread order
    float4* ckp = nullptr;
    int kc = 0;                 // contributors left before the next checkpoint
    if (FILL && THIN) {
        const uint32_t nck = valid ? ((uint32_t)a.ncontrib[pg] + (uint32_t)a.thin_k - 1u) / (uint32_t)a.thin_k : 0u;
        uint32_t inc = nck;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += o;
        }
        if (lane == kWave - 1) s_scan4[wid][0] = inc;
        __syncthreads();
        uint32_t base = 0;
        for (int w = 0; w < wid; ++w) base += s_scan4[w][0];
        const uint32_t off = base + inc - nck;
        if (valid) a.pix_ck[pg] = off;
        ckp = (float4*)a.ck + a.tile_ck_off[t] + off;
        __syncthreads();
    }

    // this thread's entry of a batch (Gaussian and record): the count pass
    // loads it one batch ahead, so that the loads overlap the blending of the
    // batch before; the fill pass (short of registers) loads the Gaussians
    // and per-block counts one batch ahead and, at the batch's start, only
    // the records of entries with pairs
    uint32_t nx_g = 0u;
    double nx_rec[10];
    auto fetch = [&](int64_t bb) {
        if (bb + tid < ke) {
            nx_g = a.vals[bb + tid];
            const int64_t r = (int64_t)v * a.N + nx_g;
#pragma unroll
            for (int i = 0; i < 10; ++i) nx_rec[i] = a.rec64[r * kRecStride + i];
        }
    };
    // fill: the batch's Gaussians and per-block counts one batch ahead
    uint32_t nf_g = 0u, nf_cnt = 0u;
    auto fetch_fill = [&](int64_t bb) {
        nf_cnt = 0u;
        if (bb + tid < ke) {
            nf_g = a.vals[bb + tid];
            nf_cnt = a.entry_cnt[bb + tid];
        }
    };
    if (FILL) fetch_fill(ks);
    if (!FILL) fetch(ks);
    for (int64_t b0 = ks; b0 < ke; b0 += kBlock) {
        if (FILL && (uint32_t)(b0 - ks) >= stop) done = true;
        if (__syncthreads_and(done ? 1 : 0)) break;
        const int nb = (int)(ke - b0 < kBlock ? ke - b0 : kBlock);
        uint32_t ecnt = 0;
        if (FILL) {
            if (tid < nb) {
                const uint32_t gi = nf_g;
                const int64_t r = (int64_t)v * a.N + gi;
                s_g[tid] = gi;
                ecnt = nf_cnt;
                if (ecnt != 0u) {
#pragma unroll
                    for (int i = 0; i < 10; ++i) s_rec[i][tid] = a.rec64[r * kRecStride + i];
                }
            }
            fetch_fill(b0 + kBlock);
        } else {
            if (tid < nb) {
                s_g[tid] = nx_g;
#pragma unroll
                for (int i = 0; i < 10; ++i) s_rec[i][tid] = nx_rec[i];
            }
            fetch(b0 + kBlock);
        }
        int nact = 0;
        if (FILL) {
            // per entry and block the padded piece, placed in depth order
            // (one thread per block); a block-wide exclusive scan gives each
            // active entry its segment index
            const uint32_t c = ecnt;
            s_cnt[tid] = c;
            uint32_t cw[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) cw[w] = (c >> (8 * w)) & 0xFFu;
            const uint32_t tot = cw[0] + cw[1] + cw[2] + cw[3];
            const uint32_t vac = tot > 0 ? 1u : 0u;
            uint32_t iac = vac;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t oac = __shfl_up(iac, off, kWave);
                if (lane >= off) iac += oac;
            }
            if (lane == kWave - 1) s_scan4[wid][2] = iac;
            __syncthreads();
            {
                // wave w places block w's pieces of the batch, 64 at a time
                uint32_t e = s_blk[wid];
                for (int j0 = 0; j0 < nb; j0 += kWave) {
                    const int j = j0 + lane;
                    const uint32_t cj = j < nb ? (s_cnt[j] >> (8 * wid)) & 0xFFu : 0u;
                    const uint32_t len = THIN ? (cj ? 1u : 0u) : pad8(cj);
                    uint32_t gap, off;
                    e = place_wave(e, len, !THIN, gap, off);
                    if (j < nb) {
                        s_egap[j][wid] = s_bbase[wid] + gap;
                        s_eoff[j][wid] = s_bbase[wid] + off;
                    }
                }
                if (lane == 0) s_blk[wid] = e;
            }
            uint32_t bac = 0, tac = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (w < wid) bac += s_scan4[w][2];
                tac += s_scan4[w][2];
            }
            const uint32_t eseg = s_run[1] + bac + iac - vac;
            if (tid < nb && vac) s_act[bac + iac - vac] = (uint16_t)tid;
            nact = (int)tac;
            __syncthreads();
            uint32_t eoff[NW], egap[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                eoff[w] = s_eoff[tid][w];
                egap[w] = s_egap[tid][w];
            }
            if (tid < nb) s_eseg[tid] = (uint32_t)(seg_base + eseg);
            if (tid < nb) {
                if (tot > 0 && seg_base + eseg < seg_end) {
                    const int64_t s = seg_base + eseg;
                    const uint32_t gi = s_g[tid];
                    const int64_t gvkey = (int64_t)gi * a.V + v;
                    const uint32_t gv = (uint32_t)a.gv_idx[gvkey];
                    a.seg_gv[s] = gv;
                    a.seg_f[0 * a.seg_stride + s] = (float)(s_rec[0][tid] - (double)(tx * a.TW));
                    a.seg_f[1 * a.seg_stride + s] = (float)(s_rec[1][tid] - (double)(ty * a.TH));
                    a.seg_f[2 * a.seg_stride + s] = (float)s_rec[2][tid];
                    a.seg_f[3 * a.seg_stride + s] = (float)s_rec[3][tid];
                    a.seg_f[4 * a.seg_stride + s] = (float)s_rec[4][tid];
                    a.seg_f[5 * a.seg_stride + s] = (float)s_rec[5][tid];
                    if (THIN) {
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) a.seg_f[(6 + ch) * a.seg_stride + s] = (float)s_rec[7 + ch][tid];
                    }
                    const uint32_t slot = atomicAdd(&a.gv_cursor[gv], 1u);
                    if (a.gv_segoff[gvkey] + slot < a.gv_segoff[gvkey + 1]) a.gv_segs[a.gv_segoff[gvkey] + slot] = (uint32_t)s;
                    typename S::word* zT = (typename S::word*)a.pT;
                    typename S::word* zD = (typename S::word*)a.pD;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        if (THIN || cw[w] == 0) continue;
                        // the piece's aligned runs (and those of the gap before
                        // it) -> this segment; the gap and the piece's last,
                        // partial run get zero T words (no pair) here, and the
                        // pairs of that run are written over them after the
                        // barrier below
                        const int64_t qg = pair_base + egap[w];
                        const int64_t q0 = pair_base + eoff[w];
                        const int64_t q1 = min(q0 + (int64_t)pad8(cw[w]), pair_end);
                        const int64_t qz = q0 + (int64_t)(cw[w] & ~7u);
                        for (int64_t r = qg >> 3; r < (q1 >> 3); ++r) a.run_seg[r] = (uint32_t)s;
                        for (int64_t q = qg; q < q1; ++q) {
                            if (q >= q0 && q < qz) continue;
                            zT[q] = 0;
                            zD[q] = 0;
                            zD[a.pair_stride + q] = 0;
                            zD[2 * a.pair_stride + q] = 0;
                            a.ppix[q] = 0;
                        }
                    }
                }
            }
            __syncthreads();
            if (tid == 0) s_run[1] += tac;
        }
        __syncthreads();

        // the count pass takes every entry; the fill pass only the entries
        // with pairs in this wave's block (a key without pairs changes no
        // pixel's blend; where it saturates a pixel, the stored stop does)
        const int n_it = FILL ? nact : nb;
        for (int k = 0; k < n_it; ++k) {
            const int j = FILL ? (int)s_act[k] : k;
            if (FILL) {
                if (((s_cnt[j] >> (8 * wid)) & 0xFFu) == 0u) continue;
                if ((uint32_t)(b0 - ks) + (uint32_t)j >= stop) done = true;
            }
            bool contrib = false;
            double alpha = 0.0, a_raw = 0.0, Tn = T;
            if (!done) {
                const double dx = pxc - s_rec[0][j], dy = pyc - s_rec[1][j];
                const double A = s_rec[2][j], B = s_rec[3][j], C = s_rec[4][j];
                const double power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
                if (power <= 0.0 && power >= s_rec[6][j] - lmargin) {
                    a_raw = s_rec[5][j] * exp(power);
                    alpha = a_raw < kAlphaMax ? a_raw : kAlphaMax;
                    if (alpha >= kAlphaMin) {
                        Tn = T * (1.0 - alpha);
                        if (Tn < kTMin) {
                            done = true;
                            if (!FILL) stop = (uint32_t)(b0 - ks) + (uint32_t)j;
                        } else {
                            contrib = true;
                        }
                    }
                }
            }
            // per-block contributor counts: a build's count pass and the fill
            // pass (renders need none)
            const uint64_t bal = (FILL || a.layout) ? __ballot(contrib) : 0ull;
            if (!FILL && a.layout) {
                if (lane == 0) s_wc[j][wid] = (uint8_t)__popcll(bal);
            }
            if (FILL && THIN) {
                const uint64_t cbal = __ballot(contrib && a_raw > kAlphaMax);
                if (lane == 0 && bal != 0ull) {
                    const int64_t q = pair_base + s_eoff[j][wid];
                    if (q < pair_end) {
                        a.piece_seg[q] = s_eseg[j];
                        a.piece_mask[q] = bal;
                        a.piece_cmask[q] = cbal;
                    }
                }
                if (contrib) {
                    if (kc == 0) {   // blend state in front of contributors 0, K, 2K, ...
                        ckp[cnt / a.thin_k] = make_float4((float)T, (float)(Ch0 - acc0), (float)(Ch1 - acc1),
                                                          (float)(Ch2 - acc2));
                        kc = a.thin_k;
                    }
                    --kc;
                }
            }
            if (contrib) {
                const double w = alpha * T;
                const double c0 = s_rec[7][j], c1 = s_rec[8][j], c2 = s_rec[9][j];
                acc0 += c0 * w;
                acc1 += c1 * w;
                acc2 += c2 * w;
                if (FILL && !THIN) {
                    // the pair's place in its piece, rotated within its run of
                    // 8 by the segment: lanes of the product passes that take
                    // runs of different splats at once then hit different
                    // pixels at each step
                    const uint32_t rank = (uint32_t)__popcll(bal & lanemask_lt());
                    const uint32_t pos = (rank & ~7u) | ((rank + s_eseg[j]) & 7u);
                    const uint32_t within = s_eoff[j][wid] + pos;         // slot in the tile
                    const int64_t slot = pair_base + within;
                    if (within < blk_end) {   // always true when both passes agree
                        const double inv = 1.0 / (1.0 - alpha);
                        const float D0 = (float)(T * c0 - (Ch0 - acc0) * inv);
                        const float D1 = (float)(T * c1 - (Ch1 - acc1) * inv);
                        const float D2 = (float)(T * c2 - (Ch2 - acc2) * inv);
                        typename S::word* pT = (typename S::word*)a.pT;
                        typename S::word* pD = (typename S::word*)a.pD;
                        pT[slot] = S::enc_T((float)T, rank == 0, a_raw > kAlphaMax);
                        pD[slot] = S::enc(D0);
                        pD[a.pair_stride + slot] = S::enc(D1);
                        pD[2 * a.pair_stride + slot] = S::enc(D2);
                        a.ppix[slot] = (uint8_t)(ly * a.TW + lx);   // tile-linear pixel index
                    }
                }
                T = Tn;
                ++cnt;
            }
        }
        __syncthreads();
        if (!FILL && a.layout) {
            // per-entry counts, per-block padded totals (pieces placed in
            // depth order as the fill pass places them), active entries and
            // real pairs of the batch, and the (Gaussian, view) segment counts
            uint32_t tot = 0;
            if (tid < nb) {
                uint32_t c0 = s_wc[tid][0], c1 = s_wc[tid][1], c2 = s_wc[tid][2], c3 = s_wc[tid][3];
                a.entry_cnt[b0 + tid] = c0 | (c1 << 8) | (c2 << 16) | (c3 << 24);
                tot = c0 + c1 + c2 + c3;
                if (tot > 0) atomicAdd(&a.gv_cnt[(int64_t)s_g[tid] * a.V + v], 1u);
            }
            uint32_t act = tot > 0 ? 1u : 0u, real = tot;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                act += __shfl_xor(act, off, kWave);
                real += __shfl_xor(real, off, kWave);
            }
            if (lane == 0) {
                s_scan4[wid][2] = act;
                s_scan4[wid][3] = real;
            }
            {
                // wave w: block w's padded total, pieces placed as the fill
                // pass places them
                uint32_t e = s_blk[wid];
                for (int j0 = 0; j0 < nb; j0 += kWave) {
                    const int j = j0 + lane;
                    const uint32_t c = j < nb ? (uint32_t)s_wc[j][wid] : 0u;
                    const uint32_t len = THIN ? (c ? 1u : 0u) : pad8(c);
                    uint32_t gap, off;
                    e = place_wave(e, len, !THIN, gap, off);
                }
                if (lane == 0) s_blk[wid] = e;
            }
            __syncthreads();
            if (tid == 0) {
                for (int w = 0; w < NW; ++w) {
                    s_run[1] += s_scan4[w][2];
                    s_run[2] += s_scan4[w][3];
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (!FILL) {
        double fsq = 0.0;
        if (valid) {
            a.pixC[pg] = acc0;
            a.pixC[a.n_pix + pg] = acc1;
            a.pixC[2 * a.n_pix + pg] = acc2;
            a.ncontrib[pg] = cnt;
            if (a.layout) a.pix_stop[pg] = stop;
            const int64_t ib = 3 * cam.pix_base + (int64_t)py * cam.W + px;
            const double accs[3] = {acc0, acc1, acc2};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const double tgt = a.target ? (double)a.target[ib + ch * HW] : 0.0;
                const double r = accs[ch] - tgt;
                a.resid[ib + ch * HW] = (float)r;
                fsq += r * r;
            }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) fsq += __shfl_xor(fsq, off, kWave);
        if (lane == 0) s_red[wid] = fsq;
        if (THIN) {
            uint32_t nck = valid ? ((uint32_t)cnt + (uint32_t)a.thin_k - 1u) / (uint32_t)a.thin_k : 0u;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) nck += __shfl_xor(nck, off, kWave);
            if (lane == 0) s_scan4[wid][0] = nck;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += s_red[w];
            a.fsq_part[t] = s;
            if (a.layout) {
                a.tile_pairs[t] = s_blk[0] + s_blk[1] + s_blk[2] + s_blk[3];
                for (int w = 0; w < NW; ++w) a.tile_blk[t * kTileBlocks + w] = s_blk[w];
                a.tile_segs[t] = s_run[1];
                a.tile_real[t] = s_run[2];
            }
            if (THIN && a.layout) {
                uint32_t nck = 0;
                for (int w = 0; w < NW; ++w) nck += s_scan4[w][0];
                a.tile_ck[t] = nck;
            }
        }
    }
}

// gv compaction: for every (g, v) with segments, its record index and the
// offset of its segment list; the first gv of each Gaussian.
__global__ void k_gv_compact(const uint32_t* __restrict__ gv_cnt, const uint64_t* __restrict__ gv_idx,
                             const uint64_t* __restrict__ gv_segoff, int64_t N, int V,
                             uint32_t* __restrict__ gv_rec, uint32_t* __restrict__ gv_seg_off,
                             uint32_t* __restrict__ gv_first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t NV = N * (int64_t)V;
    if (i > NV) return;
    if (i == NV) {
        gv_first[N] = (uint32_t)gv_idx[NV];
        gv_seg_off[gv_idx[NV]] = (uint32_t)gv_segoff[NV];
        return;
    }
    const int64_t g = i / V;
    const int v = (int)(i - g * V);
    if (v == 0) gv_first[g] = (uint32_t)gv_idx[i];
    if (gv_cnt[i] > 0) {
        const uint64_t k = gv_idx[i];
        gv_rec[k] = (uint32_t)((int64_t)v * N + g);
        gv_seg_off[k] = (uint32_t)gv_segoff[i];
    }
}

__global__ void k_flag_nonzero(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] > 0 ? 1u : 0u;
}

// Sort each gv's (short) segment list ascending so reductions run in a fixed order.
// Position of every segment in the (Gaussian, view)-grouped list, and the
// gv of every list entry: per-segment sums are written at their list
// position, so the per-gv reduction reads them in order.
__global__ void k_seg_pos(const uint32_t* __restrict__ gv_segs, const uint32_t* __restrict__ seg_gv, int64_t n_seg,
                          uint32_t* __restrict__ seg_pos, uint32_t* __restrict__ list_gv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_seg) return;
    const uint32_t sg = gv_segs[i];
    seg_pos[sg] = (uint32_t)i;
    list_gv[i] = seg_gv[sg];
}

__global__ void k_gv_sort(const uint32_t* __restrict__ gv_seg_off, int64_t n_gv, uint32_t* __restrict__ gv_segs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_gv) return;
    const uint32_t b = gv_seg_off[k], e = gv_seg_off[k + 1];
    for (uint32_t i = b + 1; i < e; ++i) {
        const uint32_t key = gv_segs[i];
        uint32_t j = i;
        while (j > b && gv_segs[j - 1] > key) {
            gv_segs[j] = gv_segs[j - 1];
            --j;
        }
        gv_segs[j] = key;
    }
}

}  // namespace

hipError_t launch_raster(bool fill, int dtype, int64_t n_tiles, const RasterArgs& a, hipStream_t s) {
    dim3 g((unsigned)n_tiles), b(kBlock);
    const bool thin = a.thin_k > 0;
    if (!fill) {
        if (thin) hipLaunchKernelGGL((k_raster<false, LM_CACHE_F32, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_raster<false, LM_CACHE_F32, false>), g, b, 0, s, a);
    } else if (thin) {
        hipLaunchKernelGGL((k_raster<true, LM_CACHE_F32, true>), g, b, 0, s, a);
    } else if (dtype == LM_CACHE_F32) {
        hipLaunchKernelGGL((k_raster<true, LM_CACHE_F32, false>), g, b, 0, s, a);
    } else if (dtype == LM_CACHE_BF16) {
        hipLaunchKernelGGL((k_raster<true, LM_CACHE_BF16, false>), g, b, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_raster<true, LM_CACHE_F16, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_flag_nonzero(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_flag_nonzero, dim3(grid_for(n)), dim3(kBlock), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_gv_compact(const uint32_t* gv_cnt, const uint64_t* gv_idx, const uint64_t* gv_segoff, int64_t N,
                             int V, uint32_t* gv_rec, uint32_t* gv_seg_off, uint32_t* gv_first, hipStream_t s) {
    hipLaunchKernelGGL(k_gv_compact, dim3(grid_for(N * (int64_t)V + 1)), dim3(kBlock), 0, s, gv_cnt, gv_idx,
                       gv_segoff, N, V, gv_rec, gv_seg_off, gv_first);
    return hipGetLastError();
}

hipError_t launch_gv_sort(const uint32_t* gv_seg_off, int64_t n_gv, uint32_t* gv_segs, hipStream_t s) {
    if (n_gv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gv_sort, dim3(grid_for(n_gv)), dim3(kBlock), 0, s, gv_seg_off, n_gv, gv_segs);
    return hipGetLastError();
}

hipError_t launch_seg_pos(const uint32_t* gv_segs, const uint32_t* seg_gv, int64_t n_seg, uint32_t* seg_pos,
                          uint32_t* list_gv, hipStream_t s) {
    if (n_seg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_pos, dim3(grid_for(n_seg)), dim3(kBlock), 0, s, gv_segs, seg_gv, n_seg, seg_pos, list_gv);
    return hipGetLastError();
}

}  // namespace lm
