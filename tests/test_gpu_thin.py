"""Thinned gradient cache (section 4.4, limitations: keep the gradients only
for every K-th splat along a ray and redo the alpha blending inside those
windows) against the FP64 oracle, through the C ABI.

The thinned cache stores no per-pair value: per 64-pixel block and splat a
mask of the pixels it contributes to, per pixel the blend state (T, colour
still to be blended) in front of every K-th contributor.  The products
re-blend every pair in float32, so the oracle is the same exact Jacobian as
for the full cache and the bars are the full cache's (1e-5 norm-wise per
parameter block for J p, J^T u, b, diag(J^T J), J^T J p; the PCG direction
within the oracle's own float32 sensitivity).  K = 1 stores every pair's
state, K = 8 and 32 re-blend windows of that length (32 is the paper's
example), K = 4096 re-blends whole rays from the first contributor.

Besides parity: the thinned and the full cache give the same products to
float32 rounding, two builds give bit-identical products (the per-block
moment sums are added in block order), and the thinned cache is smaller."""
import numpy as np
import pytest

from gpu_common import BLOCKS, make_problem, oracle_pcg, pcg_direction_bar, random_direction, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PROBLEMS = {
    "tiny": dict(name="tiny"),
    "tiny_sh3": dict(name="tiny", deg=3),
    "ragged": dict(name="tiny", N=1500, deg=1, subsets=[(3, 72, 40)], seed=11, tile=(16, 8)),
    "tile8": dict(name="tiny", N=1000, deg=2, subsets=[(2, 48, 48)], seed=12, tile=(8, 8)),
    "tall": dict(name="tiny", N=1500, deg=3, subsets=[(3, 60, 100)], seed=14, tile=(8, 32)),
    "wide": dict(name="tiny", N=1200, deg=3, subsets=[(2, 96, 24)], seed=13, tile=(32, 8)),
}
WINDOWS = (1, 8, 32, 4096)


@pytest.fixture(scope="module", params=list(PROBLEMS))
def prob(request):
    pr = make_problem(**PROBLEMS[request.param])
    pr["id"] = request.param
    return pr


@pytest.fixture(scope="module")
def built(prob):
    """Full cache and the thinned caches of every window, same inputs."""
    from paper_2409_12892_amd import binding as B
    x = torch.from_numpy(prob["scene"].x).cuda()
    tgt = torch.from_numpy(prob["target"].ravel()).cuda()
    print(f"[thin] building caches for problem {prob['id']}", flush=True)
    full = B.lm_build_cache(x, prob["scene"].sh_degree, prob["cams"], tgt, tile=prob["tile"])
    thin = {K: B.lm_build_cache(x, prob["scene"].sh_degree, prob["cams"], tgt, tile=prob["tile"], thin_window=K)
            for K in WINDOWS}
    torch.cuda.synchronize()
    yield dict(B=B, x=x, target=tgt, full=full, thin=thin)
    full[0].destroy()
    for c, _, _ in thin.values():
        c.destroy()


@pytest.mark.parametrize("K", WINDOWS)
def test_thin_layout(prob, built, K):
    inf = built["thin"][K][0].info()
    ref = built["full"][0].info()
    assert inf["thin_window"] == K and ref["thin_window"] == 0
    for k in ("n_keys", "n_pairs", "n_segments", "n_gv", "n_tiles"):
        assert inf[k] == ref[k], k
    n_contrib = sum(int(vw["raster"]["n_contrib"].sum()) for vw in prob["J"].views)
    assert inf["n_pairs"] == n_contrib
    # one checkpoint per K contributors of each pixel, rounded up
    n_ck = sum(int(((vw["raster"]["n_contrib"] + K - 1) // K).sum()) for vw in prob["J"].views)
    assert inf["n_checkpoints"] == n_ck
    assert inf["n_pieces"] <= inf["n_pairs"]
    assert inf["cache_bytes"] < ref["cache_bytes"]


@pytest.mark.parametrize("K", WINDOWS)
def test_thin_apply_J(prob, built, K, report):
    sc = prob["scene"]
    for block in (None, *BLOCKS.keys()):
        p = random_direction(sc.P, sc.N, seed=10, block=block)
        u = built["B"].lm_apply_J(built["thin"][K][0], torch.from_numpy(p).cuda())
        err = rel(u.cpu().numpy(), prob["J"].apply_J(p.astype(np.float64)))
        report[("thin_J_p", prob["id"], K, block or "all")] = err
        assert err < 1e-5, block


@pytest.mark.parametrize("K", WINDOWS)
def test_thin_apply_JT_and_b(prob, built, K, report):
    rng = np.random.default_rng(20)
    u = rng.normal(size=prob["J"].n_res).astype(np.float32)
    cache, b, fsq = built["thin"][K]
    g = built["B"].lm_apply_JT(cache, torch.from_numpy(u).cuda()).cpu().numpy()
    ref = prob["J"].apply_JT(u.astype(np.float64)).reshape(g.shape)
    bref = prob["J"].b(list(prob["target"])).reshape(g.shape)
    bb = b.cpu().numpy()
    for name, sl in BLOCKS.items():
        report[("thin_JT_u", prob["id"], K, name)] = rel(g[sl], ref[sl])
        report[("thin_b", prob["id"], K, name)] = rel(bb[sl], bref[sl])
        assert rel(g[sl], ref[sl]) < 1e-5, name
        assert rel(bb[sl], bref[sl]) < 1e-5, name
    F = prob["J"].residual(list(prob["target"]))
    assert float(fsq.item()) == pytest.approx(float(F @ F), rel=1e-12)


@pytest.mark.parametrize("K", WINDOWS)
def test_thin_jacobi_diag(prob, built, K, report):
    M = built["B"].lm_jacobi_diag(built["thin"][K][0]).cpu().numpy()
    ref = prob["J"].diag_JtJ().reshape(M.shape)
    for name, sl in BLOCKS.items():
        report[("thin_diag", prob["id"], K, name)] = rel(M[sl], ref[sl])
        assert rel(M[sl], ref[sl]) < 1e-5, name


@pytest.mark.parametrize("K", WINDOWS)
def test_thin_apply_JtJ_with_damping(prob, built, K, report):
    sc = prob["scene"]
    p = random_direction(sc.P, sc.N, seed=30)
    Mref = prob["J"].diag_JtJ()
    M = torch.from_numpy(Mref.astype(np.float32).reshape(sc.P, sc.N)).cuda()
    B = built["B"]
    g, jp = B.lm_apply_JtJ(built["thin"][K][0], torch.from_numpy(p).cuda(), 0.3, M, want_jp_sqnorm=True)
    ref = prob["J"].apply_JtJ(p.astype(np.float64), 0.3, Mref.astype(np.float32).astype(np.float64))
    report[("thin_JtJ_p", prob["id"], K)] = rel(g.cpu().numpy(), ref)
    assert rel(g.cpu().numpy(), ref) < 1e-5
    Jp = prob["J"].apply_J(p.astype(np.float64))
    assert float(jp.item()) == pytest.approx(float(Jp @ Jp), rel=1e-5)
    jp2 = B.lm_jp_sqnorm(built["thin"][K][0], torch.from_numpy(p).cuda())
    assert float(jp2.item()) == float(jp.item())
    # the full cache's product agrees to float32 rounding
    gf = B.lm_apply_JtJ(built["full"][0], torch.from_numpy(p).cuda(), 0.3, M)
    assert rel(g.cpu().numpy(), gf.cpu().numpy()) < 1e-5


@pytest.mark.parametrize("K", (8, 32))
def test_thin_pcg_direction(prob, built, K, report):
    cfg = prob["cfg"]
    J = prob["J"]
    b_ref, M_ref, out = oracle_pcg(J, prob["target"], cfg["lam"], cfg["n_iters"])
    B = built["B"]
    cache, b, _ = built["thin"][K]
    M = B.lm_jacobi_diag(cache)
    deltas, stats = B.lm_pcg_solve([cache], [b], [M], cfg["lam"], cfg["n_iters"])
    d = deltas[0].cpu().numpy().ravel()
    bar = pcg_direction_bar(J, b_ref, M_ref, cfg["lam"], cfg["n_iters"])
    report[("thin_pcg_delta", prob["id"], K)] = dict(err=rel(d, out["x"]), bar=bar)
    assert stats[0]["iters"] == cfg["n_iters"]
    assert rel(d, out["x"]) < bar


def test_thin_products_are_deterministic(prob, built):
    """A second thinned build gives bit-identical products (fixed order of
    every sum: per piece over the wave, per segment over blocks)."""
    B = built["B"]
    sc = prob["scene"]
    c2, b2, _ = B.lm_build_cache(built["x"], sc.sh_degree, prob["cams"], built["target"], tile=prob["tile"],
                                 thin_window=8)
    c1, b1, _ = built["thin"][8]
    assert torch.equal(b1, b2)
    p = torch.from_numpy(random_direction(sc.P, sc.N, seed=31)).cuda()
    assert torch.equal(B.lm_apply_JtJ(c1, p), B.lm_apply_JtJ(c2, p))
    assert torch.equal(B.lm_jacobi_diag(c1), B.lm_jacobi_diag(c2))
    c2.destroy()


def test_thin_rejects_unsupported(prob, built):
    import ctypes
    B = built["B"]
    sc = prob["scene"]
    with pytest.raises(RuntimeError, match="status -5"):
        B.lm_build_cache(built["x"], sc.sh_degree, prob["cams"], built["target"], tile=prob["tile"],
                         cache_dtype="bf16", thin_window=8)
    with pytest.raises(RuntimeError, match="status -1"):
        B.lm_build_cache(built["x"], sc.sh_degree, prob["cams"], built["target"], tile=prob["tile"],
                         thin_window=4097)
    cache = built["thin"][8][0]
    lib = B.load()
    code = B.EXPORT["pair_T"]
    n = lib.lm_cache_export_size(cache.handle, code)
    buf = (ctypes.c_uint8 * max(int(n), 8))()
    st = lib.lm_cache_export(cache.handle, code, buf, ctypes.c_int64(max(int(n), 0)), B._stream())
    assert st == -5


def test_thin_persistent_pcg_matches_eager(prob, built):
    """The persistent PCG kernel on a thinned cache (its 256-thread variant)
    gives the eager solve's direction to float32 rounding."""
    B = built["B"]
    cfg = prob["cfg"]
    cache, b, _ = built["thin"][8]
    M = B.lm_jacobi_diag(cache)
    out = {}
    for mode in (0, 3):
        B.lm_pcg_use_graph(mode)
        d, st = B.lm_pcg_solve([cache], [b], [M], cfg["lam"], cfg["n_iters"])
        out[mode] = (d[0].cpu().numpy(), st[0])
    B.lm_pcg_use_graph(2)
    assert out[3][1]["iters"] == out[0][1]["iters"] == cfg["n_iters"]
    assert rel(out[3][0], out[0][0]) < 1e-5
