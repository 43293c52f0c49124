"""Parity of the paper's objective on the GPU (eq. gn-loss; supplement A.4)
with the FP64 oracle, through the C ABI.

* lm_objective_terms: w, e and E of seeded image pairs (ragged views,
  views smaller than the SSIM window, both kinds) against
  oracle.objective.terms: float64 on both sides, so the bar is the float32
  rounding of w and e (relative 1e-6, plus 1e-12 of the array's largest
  value for entries that cancel) and relative 1e-12 for E.
* residual weights on a cache: J^T W J p (+ damping), diag(J^T W J),
  sum w (J p)^2, the per-Gaussian blocks and a PCG direction against the
  oracle's weighted products with the same seeded w (the plain-product bars:
  1e-5 norm-wise, 1e-4 sqrt(B_ii B_jj) per block entry, the PCG sensitivity
  bar); J p itself stays unweighted; clearing the weights restores the plain
  diagonal.
* lm_cache_objective: the objective at the cache's point against the
  oracle's terms of its own render.  The render agrees to 2e-7 absolute, so
  the L1 sign can differ only where |c - C| is below that: b's bar is 1e-5
  norm-wise plus the effect of flipping every such residual.  eps = 1e-2
  keeps the weight's slope (lambda1^3 / (4 eps^2) at worst) small enough
  for a 1e-4 bar on the weighted diagonal.
"""
import numpy as np
import pytest

from gpu_common import BLOCKS, make_problem, pcg_direction_bar, random_direction, rel
from oracle import objective as ob, precond, solve
from paper_2409_12892_amd import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _images(cams, seed):
    """Seeded image / target pairs with structure: smooth colour ramps plus
    noise, a target that is a perturbed copy, a few exactly equal pixels."""
    rng = np.random.default_rng(seed)
    ims, tgs = [], []
    for v in range(cams.V):
        W, H = int(cams.W[v]), int(cams.H[v])
        yy, xx = np.mgrid[0:H, 0:W]
        base = np.stack([0.5 + 0.4 * np.sin(0.3 * xx + ch) * np.cos(0.2 * yy - ch) for ch in range(3)])
        im = base + rng.normal(0, 0.05, size=base.shape)
        tg = im + rng.normal(0, 0.08, size=base.shape)
        eq = rng.random(size=base.shape) < 0.02
        tg[eq] = im[eq]
        ims.append(im.astype(np.float32))
        tgs.append(tg.astype(np.float32))
    return ims, tgs


def _mixed_cams():
    return sg.Cameras.concat([sg.fibonacci_cameras(1, 37, 23), sg.fibonacci_cameras(1, 64, 64),
                              sg.fibonacci_cameras(1, 5, 3), sg.fibonacci_cameras(1, 16, 17)])


def _f32(*v):
    return [float(np.float32(a)) for a in v]


def _close(gpu, ref, rtol=1e-6):
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    bound = rtol * np.abs(ref) + 1e-12 * max(np.abs(ref).max(), 1e-300)
    bad = np.abs(gpu - ref) > bound
    assert not bad.any(), (int(bad.sum()), float(np.abs(gpu - ref)[bad].max()))


@pytest.mark.parametrize("kind,eps", [(ob.OBJ_L1_SSIM, 1e-4), (ob.OBJ_L1_SSIM, 1e-2), (ob.OBJ_L2, 1e-4)])
def test_objective_terms_match_oracle(kind, eps):
    from paper_2409_12892_amd import binding as B
    cams = _mixed_cams()
    ims, tgs = _images(cams, 3)
    print(f"[gpu objective] terms kind={kind} eps={eps}", flush=True)
    img = torch.from_numpy(np.concatenate([a.ravel() for a in ims])).cuda()
    tgt = torch.from_numpy(np.concatenate([a.ravel() for a in tgs])).cuda()
    w, e, E, ws = B.lm_objective_terms(img, tgt, cams, B.objective(kind, eps=eps))
    # the C ABI takes lambda1, lambda2 and eps as float32
    ref = ob.terms_views([a.astype(np.float64) for a in ims], [a.astype(np.float64) for a in tgs], kind,
                         *_f32(ob.LAMBDA1, ob.LAMBDA2, eps))
    _close(w.cpu().numpy(), ref["w"])
    _close(e.cpu().numpy(), ref["e"])
    assert float(E.item()) == pytest.approx(ref["E"], rel=1e-12)
    # a second call on the same workspace, E only
    _, _, E2, _ = B.lm_objective_terms(img, tgt, cams, B.objective(kind, eps=eps), w=False, e=False, workspace=ws)
    assert float(E2.item()) == float(E.item())
    ws.destroy()


def test_objective_terms_identical_images_and_bad_arguments():
    from paper_2409_12892_amd import binding as B
    cams = sg.fibonacci_cameras(2, 20, 12)
    ims, _ = _images(cams, 4)
    img = torch.from_numpy(np.concatenate([a.ravel() for a in ims])).cuda()
    w, e, E, ws = B.lm_objective_terms(img, img, cams, B.objective())
    # SSIM(x, x) = 1 up to float64 rounding (the kernel's contracted
    # multiply-adds round the numerator and denominator differently)
    assert abs(float(E.item())) < 1e-12
    assert float(w.abs().max()) < 1e-12 and float(e.abs().max()) < 1e-12
    with pytest.raises(RuntimeError):
        B.lm_objective_terms(img, img, cams, B.objective(eps=0.0), workspace=ws)
    with pytest.raises(RuntimeError):
        B.lm_objective_terms(img, img, cams, B.LmObjective(7, 0.8, 0.2, 1e-4), workspace=ws)
    ws.destroy()


PROBLEMS = {
    "tiny": dict(name="tiny"),
    "ragged": dict(name="tiny", N=1500, deg=1, subsets=[(3, 72, 40)], seed=11, tile=(16, 8)),
    "wide": dict(name="tiny", N=1200, deg=3, subsets=[(2, 96, 24)], seed=13, tile=(32, 8)),
    "tall": dict(name="tiny", N=1500, deg=3, subsets=[(3, 60, 100)], seed=14, tile=(8, 32)),
    "tall16": dict(name="tiny", N=1200, deg=3, subsets=[(3, 64, 96)], seed=15, tile=(8, 16)),
}


@pytest.fixture(scope="module", params=list(PROBLEMS))
def prob(request):
    pr = make_problem(**PROBLEMS[request.param])
    pr["id"] = request.param
    return pr


@pytest.fixture(scope="module")
def gpu(prob):
    from paper_2409_12892_amd import binding as B
    x = torch.from_numpy(prob["scene"].x).cuda()
    tgt = torch.from_numpy(prob["target"].ravel()).cuda()
    print(f"[gpu objective] building cache for problem {prob['id']}", flush=True)
    cache, b, fsq = B.lm_build_cache(x, prob["scene"].sh_degree, prob["cams"], tgt, tile=prob["tile"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(40)
    w = rng.uniform(0.0, 3.0, size=prob["J"].n_res).astype(np.float32)
    return dict(B=B, x=x, target=tgt, cache=cache, b=b, fsq=fsq, w=w)


def test_weighted_products(prob, gpu, report):
    B, cache, J = gpu["B"], gpu["cache"], prob["J"]
    sc = prob["scene"]
    w = gpu["w"]
    w64 = w.astype(np.float64)
    B.lm_set_residual_weights(cache, torch.from_numpy(w).cuda())
    p = random_direction(sc.P, sc.N, seed=31)
    pt = torch.from_numpy(p).cuda()
    # J p is the colour Jacobian's product, unweighted
    u = B.lm_apply_J(cache, pt).cpu().numpy()
    assert rel(u, J.apply_J(p.astype(np.float64))) < 1e-5
    Mref = J.diag_JtJ(w64)
    M = B.lm_jacobi_diag(cache).cpu().numpy()
    for name, sl in BLOCKS.items():
        err = rel(M[sl], Mref.reshape(M.shape)[sl])
        report[("diag_weighted", prob["id"], name)] = err
        assert err < 1e-5, name
    Mf = torch.from_numpy(Mref.astype(np.float32).reshape(sc.P, sc.N)).cuda()
    g, jp = B.lm_apply_JtJ(cache, pt, 0.3, Mf, want_jp_sqnorm=True)
    ref = J.apply_JtJ(p.astype(np.float64), 0.3, Mref.astype(np.float32).astype(np.float64), w=w64)
    report[("JtWJ_p", prob["id"])] = rel(g.cpu().numpy(), ref)
    assert rel(g.cpu().numpy(), ref) < 1e-5
    assert float(jp.item()) == pytest.approx(J.Jp_sqnorm(p.astype(np.float64), w64), rel=1e-5)
    jp2 = B.lm_jp_sqnorm(cache, pt)
    assert float(jp2.item()) == float(jp.item())


def test_weighted_blocks(prob, gpu):
    B, cache, J = gpu["B"], gpu["cache"], prob["J"]
    w64 = gpu["w"].astype(np.float64)
    B.lm_set_residual_weights(cache, torch.from_numpy(gpu["w"]).cuda())
    sel = np.arange(0, prob["scene"].N, 97, dtype=np.int64)
    got = B.lm_block_jacobi(cache, torch.from_numpy(sel).cuda()).cpu().numpy()
    ref = precond.gaussian_blocks(J.weighted(w64))[sel]
    d = np.sqrt(np.maximum(np.einsum("nii->ni", ref), 0.0))
    bar = 1e-4 * d[:, :, None] * d[:, None, :] + 1e-30
    assert np.all(np.abs(got - ref) <= bar)


def test_weighted_pcg_direction(prob, gpu, report):
    B, cache, J = gpu["B"], gpu["cache"], prob["J"]
    cfg = prob["cfg"]
    w64 = gpu["w"].astype(np.float64)
    B.lm_set_residual_weights(cache, torch.from_numpy(gpu["w"]).cuda())
    Jw = J.weighted(w64)
    b_ref = J.b(list(prob["target"]))
    M_ref = Jw.diag_JtJ()
    out = solve.pcg(Jw.apply_JtJ, b_ref, M_ref, cfg["lam"], cfg["n_iters"])
    M = B.lm_jacobi_diag(cache)
    deltas, stats = B.lm_pcg_solve([cache], [gpu["b"]], [M], cfg["lam"], cfg["n_iters"])
    d = deltas[0].cpu().numpy().ravel()
    bar = pcg_direction_bar(Jw, b_ref, M_ref, cfg["lam"], cfg["n_iters"])
    report[("pcg_delta_weighted", prob["id"])] = dict(err=rel(d, out["x"]), bar=bar)
    assert rel(d, out["x"]) < bar


def test_clearing_weights_restores_plain_products(prob, gpu):
    B, cache, J = gpu["B"], gpu["cache"], prob["J"]
    B.lm_set_residual_weights(cache, torch.from_numpy(gpu["w"]).cuda())
    B.lm_jacobi_diag(cache)
    B.lm_set_residual_weights(cache, None)
    M = B.lm_jacobi_diag(cache).cpu().numpy()
    assert rel(M, J.diag_JtJ().reshape(M.shape)) < 1e-5


def test_cache_objective_matches_oracle(prob, gpu, report):
    B, cache, J = gpu["B"], gpu["cache"], prob["J"]
    eps = 1e-2
    obj = B.objective(B.OBJ_L1_SSIM, eps=eps)
    b, Ev = B.lm_cache_objective(cache, gpu["target"], obj)
    imgs = J.images()
    tgs = [t.astype(np.float64) for t in prob["target"]]
    per_view = [ob.terms(im, tg, ob.OBJ_L1_SSIM, *_f32(ob.LAMBDA1, ob.LAMBDA2, eps)) for im, tg in zip(imgs, tgs)]
    np.testing.assert_allclose(Ev.cpu().numpy(), [t["E"] for t in per_view], rtol=1e-6)
    e_ref = np.concatenate([t["e"].ravel() for t in per_view])
    w_ref = np.concatenate([t["w"].ravel() for t in per_view])
    b_ref = -J.apply_JT(e_ref)
    diff = np.concatenate([(im - tg).ravel() for im, tg in zip(imgs, tgs)])
    amb = np.abs(diff) < 1e-6
    flip = J.apply_JT(np.where(amb, ob.LAMBDA1, 0.0))
    bar = 1e-5 * np.linalg.norm(b_ref) + np.linalg.norm(flip)
    err = np.linalg.norm(b.cpu().numpy().ravel() - b_ref)
    report[("b_l1_ssim", prob["id"])] = dict(err=err / np.linalg.norm(b_ref), ambiguous=int(amb.sum()))
    assert err <= bar
    M = B.lm_jacobi_diag(cache).cpu().numpy()
    Mref = J.diag_JtJ(w_ref).reshape(M.shape)
    for name, sl in BLOCKS.items():
        assert rel(M[sl], Mref[sl]) < 1e-4, name
    # the forward-only evaluation agrees with the cache's per-view sums
    val, ws = B.lm_objective_value(gpu["x"], prob["scene"].sh_degree, prob["cams"], gpu["target"], obj,
                                   tile=prob["tile"])
    assert float(val.item()) == pytest.approx(float(Ev.sum().item()), rel=1e-12)
    ws.destroy()
    B.lm_set_residual_weights(cache, None)


def test_l2_cache_objective_is_plain_least_squares(prob, gpu):
    B, cache = gpu["B"], gpu["cache"]
    B.lm_set_residual_weights(cache, torch.from_numpy(gpu["w"]).cuda())
    obj = B.objective(B.OBJ_L2)
    b, Ev = B.lm_cache_objective(cache, gpu["target"], obj)
    assert torch.equal(b, gpu["b"])
    assert torch.equal(Ev, B.lm_cache_view_sqnorm(cache))
    M = B.lm_jacobi_diag(cache).cpu().numpy()
    assert rel(M, prob["J"].diag_JtJ().reshape(M.shape)) < 1e-5
    val, ws = B.lm_objective_value(gpu["x"], prob["scene"].sh_degree, prob["cams"], gpu["target"], obj,
                                   tile=prob["tile"])
    val2, ws = B.lm_residual_sqnorm(gpu["x"], prob["scene"].sh_degree, prob["cams"], gpu["target"],
                                    tile=prob["tile"], workspace=ws)
    assert float(val.item()) == float(val2.item())
    ws.destroy()
