"""Low-precision cache (T and dC/dalpha stored as bfloat16 or binary16,
products in float32) on the precision workload: 20,000 Gaussians, SH 0, 4
views 128x128, 16x16 tiles, about 1.3M pairs.

The oracle reference for a 16-bit cache is the exact Jacobian re-evaluated
with T and D rounded as stored (oracle Jacobian.rounded): the products of a
16-bit cache must match it within the float32 bar of the float32 cache
(1e-5 norm-wise per parameter block), and the stored words must equal the
oracle's rounded values within one unit of the type.  The error against
the exact Jacobian (the cost of the storage type) is recorded in the parity
report."""
import numpy as np
import pytest

from gpu_common import BLOCKS, make_problem, pcg_direction_bar, random_direction, rel
from oracle import jacobian, solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DTYPES = ("f32", "bf16", "f16")


@pytest.fixture(scope="module")
def prob():
    print("[gpu precision] oracle Jacobian of the precision workload", flush=True)
    return make_problem("precision")


@pytest.fixture(scope="module", params=DTYPES)
def case(request, prob):
    from paper_2409_12892_amd import binding as B
    dt = request.param
    print(f"[gpu precision] cache {dt}", flush=True)
    x = torch.from_numpy(prob["scene"].x).cuda()
    tgt = torch.from_numpy(prob["target"].ravel()).cuda()
    cache, b, fsq = B.lm_build_cache(x, prob["scene"].sh_degree, prob["cams"], tgt, cache_dtype=dt)
    Jr = prob["J"].rounded(dt)
    yield dict(B=B, dt=dt, cache=cache, b=b, Jr=Jr)
    cache.destroy()


def test_stored_values_are_the_rounded_cache(prob, case):
    cache, dt = case["cache"], case["dt"]
    J = prob["J"]
    pairs = [vw["raster"]["pairs"] for vw in J.views]
    assert cache.info()["cache_dtype"] == {"f32": 0, "bf16": 1, "f16": 2}[dt]
    assert cache.info()["n_pairs"] == J.n_pairs
    T = cache.export("pair_T")
    D = cache.export("pair_D").reshape(3, -1)
    gid = cache.export("pair_gauss")
    pix = cache.export("pair_pix")
    # match pairs by (pixel, Gaussian)
    o_pix = np.concatenate([J.row_offsets[v] // 3 + p["pixel"] for v, p in enumerate(pairs)])
    o_g = np.concatenate([p["g"] for p in pairs])
    ka = pix.astype(np.int64) * (J.N + 1) + gid
    kb = o_pix.astype(np.int64) * (J.N + 1) + o_g
    ia, ib = np.argsort(ka), np.argsort(kb)
    np.testing.assert_array_equal(ka[ia], kb[ib])
    rnd = jacobian.CACHE_ROUNDING[dt]
    oT = rnd(np.concatenate([p["T"] for p in pairs]))[ib]
    oD = rnd(np.concatenate([p["D"] for p in pairs]))[ib]
    ulp = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10}[dt]
    tiny = {"f32": 0.0, "bf16": 0.0, "f16": 2.0 ** -24}[dt]
    assert np.all(np.abs(T[ia] - oT) <= ulp * np.abs(oT) + tiny)
    assert np.all(np.abs(D[:, ia].T - oD) <= ulp * np.abs(oD) + tiny + 1e-7)


@pytest.mark.parametrize("block", list(BLOCKS))
def test_products_match_rounded_oracle(prob, case, block, report):
    B, cache, Jr, J = case["B"], case["cache"], case["Jr"], prob["J"]
    P, N = prob["scene"].P, prob["scene"].N
    p = random_direction(P, N, seed=40, block=block)
    u = B.lm_apply_J(cache, torch.from_numpy(p).cuda()).cpu().numpy().ravel()
    ref = Jr.apply_J(p.astype(np.float64))
    err = rel(u, ref)
    report[("precision_Jp", case["dt"], block)] = dict(err=err, err_vs_exact=rel(u, J.apply_J(p.astype(np.float64))))
    assert err < 1e-5
    rng = np.random.default_rng(41)
    uu = rng.normal(size=Jr.n_res).astype(np.float32)
    g = B.lm_apply_JT(cache, torch.from_numpy(uu).cuda()).cpu().numpy().reshape(P, N)
    refg = Jr.apply_JT(uu.astype(np.float64)).reshape(P, N)
    sl = BLOCKS[block]
    assert rel(g[sl], refg[sl]) < 1e-5


def test_b_diag_and_fused_product(prob, case, report):
    B, cache, Jr, J = case["B"], case["cache"], case["Jr"], prob["J"]
    P, N = prob["scene"].P, prob["scene"].N
    ref_b = Jr.b(list(prob["target"])).reshape(P, N)
    b = case["b"].cpu().numpy()
    M = B.lm_jacobi_diag(cache).cpu().numpy()
    ref_M = Jr.diag_JtJ().reshape(P, N)
    for name, sl in BLOCKS.items():
        assert rel(b[sl], ref_b[sl]) < 1e-5, name
        assert rel(M[sl], ref_M[sl]) < 1e-5, name
    p = random_direction(P, N, seed=42)
    g = B.lm_apply_JtJ(cache, torch.from_numpy(p).cuda(), lam=1e-2,
                       M=torch.from_numpy(ref_M.astype(np.float32)).cuda()).cpu().numpy().ravel()
    ref = Jr.apply_JtJ(p.astype(np.float64), 1e-2, ref_M.astype(np.float32).astype(np.float64))
    err = rel(g, ref)
    report[("precision_JtJ", case["dt"])] = dict(err=err, err_vs_exact=rel(g, J.apply_JtJ(
        p.astype(np.float64), 1e-2, ref_M.astype(np.float32).astype(np.float64))),
        diag_vs_exact=rel(M, J.diag_JtJ().reshape(P, N)))
    assert err < 1e-5


def test_pcg_direction_low_precision(prob, case, report):
    if case["dt"] == "f32":
        pytest.skip("the float32 cache's PCG parity is covered on five scenes elsewhere")
    B, cache, Jr, J = case["B"], case["cache"], case["Jr"], prob["J"]
    # occluded Gaussians of this scene have diagonals near 1e-30, where plain
    # Jacobi steps are noise; the minimum LM diagonal the LM loop uses makes
    # the solve well posed on both sides
    lam, iters, floor = 1e-2, 8, 1e-2
    b_ref = Jr.b(list(prob["target"]))
    M_ref = Jr.diag_JtJ().astype(np.float32).astype(np.float64)
    out = solve.pcg(Jr.apply_JtJ, b_ref, M_ref, lam, iters, diag_floor=floor)
    bt = torch.from_numpy(b_ref.reshape(prob["scene"].P, -1).astype(np.float32)).cuda()
    Mt = torch.from_numpy(M_ref.reshape(prob["scene"].P, -1).astype(np.float32)).cuda()
    deltas, stats = B.lm_pcg_solve([cache], [bt], [Mt], lam, iters, diag_floor=floor)
    d = deltas[0].cpu().numpy().ravel()
    bar = pcg_direction_bar(Jr, b_ref, M_ref, lam, iters, trials=2, diag_floor=floor)
    exact = solve.pcg(J.apply_JtJ, J.b(list(prob["target"])), J.diag_JtJ(), lam, iters, diag_floor=floor)["x"]
    report[("precision_pcg", case["dt"])] = dict(err=rel(d, out["x"]), bar=bar, err_vs_exact=rel(d, exact))
    assert rel(d, out["x"]) < bar
