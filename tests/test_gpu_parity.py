"""Parity of the HIP path (through the C ABI) with the FP64 oracle, float32
cache, on several seeded scenes:

  tiny      2,048 Gaussians, SH 0, 4 views 64x64, 16x16 tiles (the plain-method config)
  tiny_sh3  the same scene drawn at SH degree 3 (59 parameters)
  ragged    1,500 Gaussians, SH 1, 3 views 72x40, 16x8 tiles (partial tiles in x and y)
  tile8     1,000 Gaussians, SH 2, 2 views 48x48, 8x8 tiles
  wide      1,200 Gaussians, SH 3, 2 views 96x24, 32x8 tiles
  tall      1,500 Gaussians, SH 3, 3 views 60x100, 8x32 tiles (the shape the
            autotuner picks at the paper workload; partial tiles in x and y)
  tall16    1,200 Gaussians, SH 3, 3 views 64x96, 8x16 tiles
  dense     6,000 Gaussians, SH 1, 2 views 32x32, 16x16 tiles (850-990 splats
            with pairs per tile: more than the tile pass stages at once)
  dense_tall  the same at 8x32 tiles (up to 1,670 splats per tile)

Bars: tile binning and depth order bit-exact (each GPU tile list an
order-preserving subsequence of the oracle's 3-sigma-rectangle list, every
left-out key certified below the alpha threshold pixel by pixel); active
pair set exact; J p, J^T u,
b = -J^T F and diag(J^T J) within a norm-wise relative error of 1e-5 (per
parameter block); PCG directions within max(1e-4, the oracle's own
sensitivity to float32-sized product perturbations)."""
import numpy as np
import pytest

from gpu_common import BLOCKS, make_problem, oracle_pcg, pcg_direction_bar, random_direction, rel
from oracle import forward, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


PROBLEMS = {
    "tiny": dict(name="tiny"),
    "tiny_sh3": dict(name="tiny", deg=3),
    "ragged": dict(name="tiny", N=1500, deg=1, subsets=[(3, 72, 40)], seed=11, tile=(16, 8)),
    "tile8": dict(name="tiny", N=1000, deg=2, subsets=[(2, 48, 48)], seed=12, tile=(8, 8)),
    "wide": dict(name="tiny", N=1200, deg=3, subsets=[(2, 96, 24)], seed=13, tile=(32, 8)),
    "tall": dict(name="tiny", N=1500, deg=3, subsets=[(3, 60, 100)], seed=14, tile=(8, 32)),
    "tall16": dict(name="tiny", N=1200, deg=3, subsets=[(3, 64, 96)], seed=15, tile=(8, 16)),
    # 6,000 small Gaussians over 2 views 32x32: 850-1700 splats with pairs
    # per tile, more than the tile pass stages at once (chunked segments)
    "dense": dict(name="tiny", N=6000, deg=1, subsets=[(2, 32, 32)], seed=16, tile=(16, 16)),
    "dense_tall": dict(name="tiny", N=6000, deg=1, subsets=[(2, 32, 32)], seed=16, tile=(8, 32)),
}
# segments the tile pass stages in LDS at once (a tile with more runs chunk by chunk)
TILE_SEG_CAP = 640


@pytest.fixture(scope="module", params=list(PROBLEMS))
def prob(request):
    kw = dict(PROBLEMS[request.param])
    pr = make_problem(**kw)
    pr["id"] = request.param
    return pr


@pytest.fixture(scope="module")
def gpu(prob):
    from paper_2409_12892_amd import binding as B
    x = torch.from_numpy(prob["scene"].x).cuda()
    tgt = torch.from_numpy(prob["target"].ravel()).cuda()
    print(f"[gpu parity] building cache for problem {prob['id']}", flush=True)
    cache, b, fsq = B.lm_build_cache(x, prob["scene"].sh_degree, prob["cams"], tgt, tile=prob["tile"])
    torch.cuda.synchronize()
    return dict(B=B, x=x, target=tgt, cache=cache, b=b, fsq=fsq)


def _img_shape(prob):
    cams = prob["cams"]
    return cams.V, int(cams.H[0]), int(cams.W[0])


def test_library_loaded_is_in_tree(gpu):
    import os
    from paper_2409_12892_amd import binding
    assert os.path.dirname(binding.LIB_PATH).endswith("paper_2409_12892_amd")


def test_projection_records(prob, gpu):
    rec = gpu["cache"].export("records").reshape(prob["cams"].V, -1, 4)
    x64 = prob["scene"].x.astype(np.float64)
    for v in range(prob["cams"].V):
        pr = forward.project(x64, prob["cams"].view(v), prob["scene"].sh_degree)
        vis = pr["visible"]
        np.testing.assert_array_equal(rec[v, vis, 0], pr["y"][0][vis].astype(np.float32))
        np.testing.assert_array_equal(rec[v, vis, 1], pr["y"][1][vis].astype(np.float32))
        np.testing.assert_array_equal(rec[v, vis, 2], pr["z"][vis].astype(np.float32))
        np.testing.assert_array_equal(rec[v, vis, 3].astype(np.int64), pr["radius"][vis])


def _below_threshold_everywhere(y, g, t, TX, TW, TH, W, H):
    """alpha = o exp(power) < 1/255 at every pixel centre of tile t inside
    the image, from the oracle's float64 projection (pixel by pixel)."""
    tx, ty = t % TX, t // TX
    px = tx * TW + np.arange(TW)
    py = ty * TH + np.arange(TH)
    px, py = px[px < W] + 0.5, py[py < H] + 0.5
    dx = px[None, :] - y[0, g]
    dy = py[:, None] - y[1, g]
    power = -0.5 * (y[2, g] * dx * dx + y[4, g] * dy * dy) - y[3, g] * dx * dy
    return bool((y[5, g] * np.exp(power) < forward.ALPHA_MIN).all())


def check_tile_lists(vals, rng, J, tile):
    """Each GPU tile list is an order-preserving subsequence of the oracle's
    full 3-sigma-rectangle list (bit-exact integer binning and depth order),
    and every key the GPU leaves out is certified non-contributing by the
    oracle: the splat stays below the alpha threshold at every pixel centre
    of the tile.  Returns (oracle keys, left-out keys)."""
    t0 = 0
    n_keys = n_out = 0
    for v, vw in enumerate(J.views):
        lists = vw["bins"]["lists"]
        y = np.real(vw["proj"]["y"])
        TX = vw["bins"]["TX"]
        W, H = vw["cam"]["W"], vw["cam"]["H"]
        TW, TH = tile
        for t, lst in enumerate(lists):
            got = vals[rng[t0 + t]:rng[t0 + t + 1]].astype(np.int64)
            keep = np.isin(lst, got)
            np.testing.assert_array_equal(got, lst[keep], err_msg=f"view {v} tile {t}: not a subsequence")
            for g in lst[~keep]:
                assert _below_threshold_everywhere(y, g, t, TX, TW, TH, W, H), f"view {v} tile {t}: dropped {g}"
            n_keys += len(lst)
            n_out += int((~keep).sum())
        t0 += len(lists)
    assert rng[-1] == len(vals)
    return n_keys, n_out


def test_binning_and_sort_bit_exact(prob, gpu, report):
    """Integer binning and depth order against the oracle's 3-sigma-rectangle
    lists; the keys the GPU leaves out (tiles where the splat cannot reach
    the alpha threshold) are certified pixel by pixel."""
    assert gpu["cache"].info()["tile_w"] == prob["tile"][0]
    vals = gpu["cache"].export("sorted_values")
    rng = gpu["cache"].export("tile_ranges")
    n_keys, n_out = check_tile_lists(vals, rng, prob["J"], prob["tile"])
    assert gpu["cache"].info()["n_keys"] == n_keys - n_out
    report[("binning_left_out_fraction", prob["id"])] = n_out / max(n_keys, 1)


def test_render_and_contributors(prob, gpu):
    V, H, W = _img_shape(prob)
    img = gpu["cache"].export("image").reshape(V, 3, H, W)
    nc = gpu["cache"].export("ncontrib").reshape(V, H, W)
    for v, vw in enumerate(prob["J"].views):
        np.testing.assert_allclose(img[v], vw["raster"]["image"], rtol=0, atol=2e-7)
        np.testing.assert_array_equal(nc[v], vw["raster"]["n_contrib"])
    res = gpu["cache"].export("residual")
    F = prob["J"].residual(list(prob["target"]))
    np.testing.assert_allclose(res, F, rtol=0, atol=2e-7)
    assert float(gpu["fsq"].item()) == pytest.approx(float(F @ F), rel=1e-12)


def test_cache_pairs_match_oracle(prob, gpu):
    c = gpu["cache"]
    pix = c.export("pair_pix").astype(np.int64)
    gid = c.export("pair_gauss").astype(np.int64)
    T = c.export("pair_T")
    D = c.export("pair_D").reshape(3, -1)
    V, H, W = _img_shape(prob)
    HW = H * W
    o_pix, o_g, o_T, o_D = [], [], [], []
    for v, vw in enumerate(prob["J"].views):
        p = vw["raster"]["pairs"]
        o_pix.append(p["pixel"] + v * HW)
        o_g.append(p["g"])
        o_T.append(p["T"])
        o_D.append(p["D"])
    o_pix, o_g = np.concatenate(o_pix), np.concatenate(o_g)
    o_T, o_D = np.concatenate(o_T), np.concatenate(o_D)
    assert len(pix) == len(o_pix)
    key_gpu = pix * 10_000_000 + gid
    key_or = o_pix * 10_000_000 + o_g
    ig, io = np.argsort(key_gpu), np.argsort(key_or)
    np.testing.assert_array_equal(key_gpu[ig], key_or[io])
    np.testing.assert_allclose(T[ig], o_T[io], rtol=1e-7, atol=0)
    np.testing.assert_allclose(D[:, ig].T, o_D[io], rtol=0, atol=1e-6)


def test_tile_segments_count_the_splats_with_pairs(prob, gpu):
    """Per tile, the segments (splats with at least one pair in the tile)
    equal the oracle's distinct Gaussians among the tile's pairs."""
    seg = np.diff(gpu["cache"].export("tile_segments"))
    V, H, W = _img_shape(prob)
    TW, TH = prob["tile"]
    TX, TY = -(-W // TW), -(-H // TH)
    N = prob["scene"].N
    counts = np.zeros(V * TX * TY, np.int64)
    for v, vw in enumerate(prob["J"].views):
        p = vw["raster"]["pairs"]
        y, x = p["pixel"] // W, p["pixel"] % W
        t = v * TX * TY + (y // TH) * TX + x // TW
        u = np.unique(t.astype(np.int64) * (N + 1) + p["g"])
        np.add.at(counts, u // (N + 1), 1)
    np.testing.assert_array_equal(seg, counts)
    assert seg.sum() == gpu["cache"].info()["n_segments"]
    if prob["id"] == "dense":
        assert seg.min() > TILE_SEG_CAP             # every tile in two segment chunks
    if prob["id"] == "dense_tall":
        assert seg.max() > 2 * TILE_SEG_CAP         # three chunks in the middle tiles


@pytest.mark.parametrize("block", [None, *BLOCKS.keys()])
def test_apply_J(prob, gpu, block, report):
    sc = prob["scene"]
    p = random_direction(sc.P, sc.N, seed=10, block=block)
    u = gpu["B"].lm_apply_J(gpu["cache"], torch.from_numpy(p).cuda())
    ref = prob["J"].apply_J(p.astype(np.float64))
    err = rel(u.cpu().numpy(), ref)
    report[("J_p", prob["id"], block or "all")] = err
    assert err < 1e-5


@pytest.mark.parametrize("block", [None, *BLOCKS.keys()])
def test_apply_JT(prob, gpu, block, report):
    rng = np.random.default_rng(20)
    u = rng.normal(size=prob["J"].n_res).astype(np.float32)
    g = gpu["B"].lm_apply_JT(gpu["cache"], torch.from_numpy(u).cuda()).cpu().numpy()
    ref = prob["J"].apply_JT(u.astype(np.float64)).reshape(g.shape)
    sl = slice(None) if block is None else BLOCKS[block]
    err = rel(g[sl], ref[sl])
    report[("JT_u", prob["id"], block or "all")] = err
    assert err < 1e-5


def test_b_is_minus_JT_F(prob, gpu, report):
    ref = prob["J"].b(list(prob["target"])).reshape(prob["scene"].P, -1)
    b = gpu["b"].cpu().numpy()
    for name, sl in BLOCKS.items():
        report[("b", prob["id"], name)] = rel(b[sl], ref[sl])
        assert rel(b[sl], ref[sl]) < 1e-5, name


def test_jacobi_diag(prob, gpu, report):
    M = gpu["B"].lm_jacobi_diag(gpu["cache"]).cpu().numpy()
    ref = prob["J"].diag_JtJ().reshape(M.shape)
    for name, sl in BLOCKS.items():
        report[("diag", prob["id"], name)] = rel(M[sl], ref[sl])
        assert rel(M[sl], ref[sl]) < 1e-5, name


def test_apply_JtJ_fused_with_damping(prob, gpu, report):
    sc = prob["scene"]
    p = random_direction(sc.P, sc.N, seed=30)
    Mref = prob["J"].diag_JtJ()
    M = torch.from_numpy(Mref.astype(np.float32).reshape(sc.P, sc.N)).cuda()
    g, jp = gpu["B"].lm_apply_JtJ(gpu["cache"], torch.from_numpy(p).cuda(), 0.3, M, want_jp_sqnorm=True)
    ref = prob["J"].apply_JtJ(p.astype(np.float64), 0.3, Mref.astype(np.float32).astype(np.float64))
    report[("JtJ_p", prob["id"])] = rel(g.cpu().numpy(), ref)
    assert rel(g.cpu().numpy(), ref) < 1e-5
    Jp = prob["J"].apply_J(p.astype(np.float64))
    assert float(jp.item()) == pytest.approx(float(Jp @ Jp), rel=1e-5)
    # the J-only entry point gives the same norm (same tile partials, same order)
    jp2 = gpu["B"].lm_jp_sqnorm(gpu["cache"], torch.from_numpy(p).cuda())
    assert float(jp2.item()) == float(jp.item())


# sub-pixel splats behind others have Jacobi diagonals near 1e-29: Algorithm
# 1 without a minimum diagonal then steps by b / M with b itself a float32
# rounding residue (the oracle's direction is 2.6e11 on one such parameter);
# the dense problems check PCG with the minimum diagonal instead
# (test_pcg_with_diag_floor)
UNFLOORED_PCG_SKIP = {"dense", "dense_tall"}


def test_pcg_direction(prob, gpu, report):
    if prob["id"] in UNFLOORED_PCG_SKIP:
        pytest.skip("Jacobi diagonals near 1e-29 (sub-pixel occluded splats): checked with a minimum diagonal")
    cfg = prob["cfg"]
    J = prob["J"]
    b_ref, M_ref, out = oracle_pcg(J, prob["target"], cfg["lam"], cfg["n_iters"])
    B = gpu["B"]
    M = B.lm_jacobi_diag(gpu["cache"])
    deltas, stats = B.lm_pcg_solve([gpu["cache"]], [gpu["b"]], [M], cfg["lam"], cfg["n_iters"])
    d = deltas[0].cpu().numpy().ravel()
    assert stats[0]["iters"] == cfg["n_iters"] and stats[0]["status"] == 0
    bar = pcg_direction_bar(J, b_ref, M_ref, cfg["lam"], cfg["n_iters"])
    report[("pcg_delta_10it", prob["id"])] = dict(err=rel(d, out["x"]), bar=bar)
    assert rel(d, out["x"]) < bar
    np.testing.assert_allclose(stats[0]["history"], out["history"], rtol=1e-3)


def test_pcg_paper_stopping_rule(prob, gpu, report):
    """Algorithm 1's break: ||r||^2 < 0.01 ||b||^2 ends the loop on the device."""
    if prob["id"] in UNFLOORED_PCG_SKIP:
        pytest.skip("Jacobi diagonals near 1e-29 (sub-pixel occluded splats): checked with a minimum diagonal")
    J = prob["J"]
    _, _, out = oracle_pcg(J, prob["target"], 1e-2, 50, tol=0.01, tol_mode=solve.TOL_PAPER_SQUARED)
    B = gpu["B"]
    M = B.lm_jacobi_diag(gpu["cache"])
    deltas, stats = B.lm_pcg_solve([gpu["cache"]], [gpu["b"]], [M], 1e-2, 50, tol=0.01,
                                   tol_mode=B.TOL_PAPER_SQUARED)
    assert stats[0]["iters"] == out["iters"]
    assert stats[0]["history"][-1] < 0.01
    np.testing.assert_allclose(stats[0]["history"], out["history"], rtol=1e-3)
    err = rel(deltas[0].cpu().numpy().ravel(), out["x"])
    bar = pcg_direction_bar(J, J.b(list(prob["target"])), J.diag_JtJ(), 1e-2, out["iters"])
    report[("pcg_paper_rule_delta", prob["id"])] = dict(err=err, iters=int(out["iters"]), bar=bar)
    assert err < bar


def test_pcg_with_diag_floor(prob, gpu, report):
    """Minimum LM diagonal: positive diagonal entries below the floor are raised
    to it in both the damping and the preconditioner (oracle reading of the
    same option)."""
    J = prob["J"]
    b = J.b(list(prob["target"]))
    M = J.diag_JtJ()
    floor = float(np.quantile(M[M > 0], 0.2))
    out = solve.pcg(J.apply_JtJ, b, M, 1e-2, 10, diag_floor=floor)
    B = gpu["B"]
    Mg = B.lm_jacobi_diag(gpu["cache"])
    deltas, stats = B.lm_pcg_solve([gpu["cache"]], [gpu["b"]], [Mg], 1e-2, 10, diag_floor=floor)
    err = rel(deltas[0].cpu().numpy().ravel(), out["x"])
    bar = pcg_direction_bar(J, b, M, 1e-2, 10, diag_floor=floor)
    report[("pcg_delta_floor_10it", prob["id"])] = dict(err=err, bar=bar)
    assert err < bar


def test_combine_subsets(gpu):
    B = gpu["B"]
    rng = np.random.default_rng(5)
    ds = [rng.normal(size=1000).astype(np.float32) for _ in range(3)]
    Ms = [np.abs(rng.normal(size=1000)).astype(np.float32) for _ in range(3)]
    for m in Ms:
        m[rng.integers(0, 1000, 100)] = 0.0
    Ms[0][:5] = Ms[1][:5] = Ms[2][:5] = 0.0
    out = B.lm_combine_subsets([torch.from_numpy(d).cuda() for d in ds], [torch.from_numpy(m).cuda() for m in Ms])
    ref = solve.combine_subsets(ds, Ms)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
    assert np.all(out.cpu().numpy()[:5] == 0)


def test_render_entry_point(prob, gpu):
    img = gpu["B"].lm_render(gpu["x"], prob["scene"].sh_degree, prob["cams"], tile=prob["tile"]).cpu().numpy()
    ref = np.concatenate([vw["raster"]["image"].ravel() for vw in prob["J"].views])
    np.testing.assert_allclose(img, ref, rtol=0, atol=2e-7)


def test_rebuild_reuses_cache_and_is_deterministic(prob, gpu):
    B = gpu["B"]
    c2, b2, _ = B.lm_build_cache(gpu["x"], prob["scene"].sh_degree, prob["cams"], gpu["target"], tile=prob["tile"])
    assert np.array_equal(c2.export("sorted_values"), gpu["cache"].export("sorted_values"))
    assert torch.equal(b2, gpu["b"]) or rel(b2.cpu().numpy(), gpu["b"].cpu().numpy()) < 1e-6
    c3, b3, _ = B.lm_build_cache(gpu["x"], prob["scene"].sh_degree, prob["cams"], gpu["target"], cache=c2,
                                 tile=prob["tile"])
    assert np.array_equal(c3.export("pair_T"), gpu["cache"].export("pair_T"))
    c2.destroy()
