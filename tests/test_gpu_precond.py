"""Learned diagonal preconditioner on the GPU against the oracle
(oracle/precond.py): pair coverage (exact counts), the per-Gaussian J^T J
blocks, the row-sum targets, the features, the perceptron's forward pass,
its gradient and one Adam step; then GPU training and the preconditioner's
effect on PCG iterations on a held-out scene.

Tolerances:
* blocks: every entry within 1e-4 sqrt(B_ii B_jj).  An entry is a sum over
  pairs and colour channels of products of two Jacobian entries, so by
  Cauchy-Schwarz the sum of the magnitudes of its terms is at most
  sqrt(B_ii B_jj); float32 accumulation over a few hundred terms per
  (Gaussian, view) plus the float32 cache values stay far below 1e-4 of it.
* targets: t within 1e-3 (a relative error of at most 1e-4 in D and the row
  sum; the shrinkage averages such errors), mask identical.
* features: 1e-4 on the centred logs (relative 1e-5 in M), 1e-6 on the two
  features taken from x.
* perceptron: weights and inputs are rounded to bfloat16 before both sides
  see them, so the GPU products are exact up to float32 accumulation and the
  bfloat16 rounding of the hidden activations (relative 2^-9 each).  The
  forward bar propagates that rounding through the layers with the oracle's
  own activations (|gelu'| <= 1.13); the gradient bar is 8 roundings of
  2^-8 of the same products taken in absolute value."""
import math

import numpy as np
import pytest

from gpu_common import make_problem
from oracle import jacobian, precond

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LAM, FLOOR = 1e-2, 1e-2
U = 2.0 ** -8          # bfloat16 relative rounding bound, with a factor 2 of margin


@pytest.fixture(scope="module", params=["tiny", "sh3"])
def prob(request):
    if request.param == "tiny":
        print("[gpu precond] oracle Jacobian of the tiny workload", flush=True)
        p = make_problem("tiny")
    else:
        print("[gpu precond] oracle Jacobian of a 600-Gaussian SH-3 scene, 2 views 64x64", flush=True)
        p = make_problem("tiny", N=600, subsets=[(2, 64, 64)], seed=35, deg=3)
    p["id"] = request.param
    from paper_2409_12892_amd import binding as B
    x = torch.from_numpy(p["scene"].x).cuda()
    tgt = torch.from_numpy(p["target"].ravel()).cuda()
    cache, b, _ = B.lm_build_cache(x, p["scene"].sh_degree, p["cams"], tgt)
    p.update(B=B, x=x, cache=cache, blocks=precond.gaussian_blocks(p["J"]))
    yield p
    cache.destroy()


def oracle_coverage(J, N):
    return np.bincount(np.concatenate([vw["raster"]["pairs"]["g"] for vw in J.views]), minlength=N)


def test_pair_coverage_is_exact(prob):
    cov = prob["B"].lm_pair_coverage(prob["cache"]).cpu().numpy()
    np.testing.assert_array_equal(cov, oracle_coverage(prob["J"], prob["scene"].N).astype(np.float32))


def test_blocks_match_oracle(prob, report):
    N, P = prob["scene"].N, prob["scene"].P
    sel = torch.arange(N, device="cuda", dtype=torch.int64)
    got = prob["B"].lm_block_jacobi(prob["cache"], sel).double().cpu().numpy()
    ref = prob["blocks"]
    d = np.einsum("kii->ki", ref)
    scale = np.sqrt(np.maximum(d[:, :, None] * d[:, None, :], 0.0))
    err = np.abs(got - ref)
    worst = float(np.max(err / np.maximum(scale, 1e-300)))
    report[("precond_blocks", prob["id"])] = worst
    assert np.all(err <= 1e-4 * scale + 1e-30), worst
    # a selection in any order, with repeats
    pick = np.array([5, 0, N - 1, 5, N // 2], np.int64)
    got2 = prob["B"].lm_block_jacobi(prob["cache"], torch.from_numpy(pick).cuda()).double().cpu().numpy()
    np.testing.assert_array_equal(got2, got[pick])


@pytest.mark.parametrize("shrink", [1.0, 0.5, 0.0])
def test_targets_match_oracle(prob, shrink, report):
    t, m = prob["B"].lm_precond_targets(prob["cache"], LAM, FLOOR, shrink=shrink)
    t, m = t.double().cpu().numpy(), m.cpu().numpy()
    tr, mr = precond.targets(prob["blocks"], LAM, diag_floor=FLOOR, beta=shrink)
    np.testing.assert_array_equal(m, mr.astype(np.float32))
    report[("precond_targets", prob["id"], shrink)] = float(np.max(np.abs(t - tr)))
    assert np.max(np.abs(t - tr)) <= 1e-3
    assert np.all(t[~mr] == 0)


def test_features_match_oracle(prob, report):
    B, cache = prob["B"], prob["cache"]
    M = B.lm_jacobi_diag(cache)
    f = B.lm_precond_features(cache, prob["x"], M).double().cpu().numpy()
    N = prob["scene"].N
    Mr = prob["J"].diag_JtJ().reshape(prob["scene"].P, N)
    fr = precond.features(Mr, oracle_coverage(prob["J"], N), prob["scene"].x)
    err = np.abs(f - fr)
    report[("precond_features", prob["id"])] = float(err.max())
    assert err[:6].max() <= 1e-4
    assert err[6:].max() <= 1e-6


# ---- perceptron -----------------------------------------------------------------

def bf16_params(p_out, seed):
    rng = np.random.default_rng(seed)
    par = precond.init_params(p_out, seed=seed)
    for k in par:                                    # non-zero biases, larger output weights
        par[k] = par[k] + 0.05 * rng.normal(size=par[k].shape)
    return {k: jacobian.round_bf16(v) for k, v in par.items()}


def pack(par, p_out):
    from paper_2409_12892_amd import binding as B
    w = np.zeros(B.MLP_PARAMS, np.float32)
    for k, (off, shape) in B.MLP_OFFSETS.items():
        a = np.zeros(shape)
        if k == "W3":
            a[:, :p_out] = par[k]
        elif k == "b3":
            a[:p_out] = par[k]
        else:
            a[...] = par[k]
        w[off:off + a.size] = a.reshape(-1)
    return torch.from_numpy(w).cuda()


def unpack_grad(g, p_out):
    from paper_2409_12892_amd import binding as B
    d = B.mlp_unpack(g)
    d["W3"] = d["W3"][:, :p_out]
    d["b3"] = d["b3"][:p_out]
    return d


def forward_bar(par, f):
    """First-order bound on |s_gpu - s| from the bfloat16 rounding of h1 and
    h2 (relative U each) plus float32 accumulation, from the oracle's own
    intermediate values."""
    s, (X, z1, h1, z2, h2) = precond.forward(par, f)
    f32 = 2.0 ** -22
    e_h1 = U * np.abs(h1) + 1.13 * f32 * (np.abs(X) @ np.abs(par["W1"]) + np.abs(par["b1"]))
    e_z2 = e_h1 @ np.abs(par["W2"]) + f32 * (np.abs(h1) @ np.abs(par["W2"]) + np.abs(par["b2"]))
    e_h2 = 1.13 * e_z2 + U * np.abs(h2)
    e_s = e_h2 @ np.abs(par["W3"]) + f32 * (np.abs(h2) @ np.abs(par["W3"]) + np.abs(par["b3"]))
    return s, 2.0 * e_s.T + 1e-7


@pytest.mark.parametrize("p_out,n", [(59, 1237), (14, 16), (7, 1), (64, 333)])
def test_mlp_forward_matches_oracle(p_out, n, report):
    from paper_2409_12892_amd import binding as B
    rng = np.random.default_rng(60 + p_out)
    par = bf16_params(p_out, 61)
    f = jacobian.round_bf16(rng.normal(size=(8, n)) * 1.5)
    s_ref, bar = forward_bar(par, f)
    s, sc, nf = B.lm_mlp_forward(pack(par, p_out), torch.from_numpy(f.astype(np.float32)).cuda(), p_out)
    s, sc = s.double().cpu().numpy(), sc.double().cpu().numpy()
    err = np.abs(s - s_ref)
    report[("mlp_forward", p_out, n)] = float(np.max(err / bar))
    assert np.all(err <= bar), float(np.max(err / bar))
    np.testing.assert_allclose(sc, np.exp(np.clip(s, -4, 4)), rtol=2e-6)
    assert int(nf.item()) == 0


def test_mlp_forward_non_finite_input_falls_back_to_jacobi():
    from paper_2409_12892_amd import binding as B
    par = bf16_params(11, 62)
    f = np.zeros((8, 40), np.float32)
    f[3, 7] = np.nan
    s, sc, nf = B.lm_mlp_forward(pack(par, 11), torch.from_numpy(f).cuda(), 11)
    sc = sc.cpu().numpy()
    assert np.all(sc[:, 7] == 1.0)
    assert int(nf.item()) == 11
    assert np.all(np.isfinite(sc)) and np.all(sc[:, 6] > 0)


def grad_bar(par, f, t, mask, e_s):
    """|gradient| products in absolute value with the forward error folded
    into the output residual; the bar is 8 U of it."""
    s, (X, z1, h1, z2, h2) = precond.forward(par, f)
    m = mask.astype(np.float64)
    cnt = max(m.sum(), 1.0)
    ds = (2.0 / cnt) * (np.abs(s - t) + e_s) * m
    ds = ds.T
    gp1 = np.abs(precond.gelu_grad(z1))
    gp2 = np.abs(precond.gelu_grad(z2))
    a = {"W3": np.abs(h2).T @ ds, "b3": ds.sum(axis=0)}
    dz2 = (ds @ np.abs(par["W3"]).T) * gp2
    a["W2"], a["b2"] = np.abs(h1).T @ dz2, dz2.sum(axis=0)
    dz1 = (dz2 @ np.abs(par["W2"]).T) * gp1
    a["W1"], a["b1"] = np.abs(X).T @ dz1, dz1.sum(axis=0)
    return {k: 8 * U * v + 1e-9 for k, v in a.items()}


@pytest.mark.parametrize("p_out,n", [(59, 2000), (14, 77)])
def test_mlp_gradient_and_adam_step_match_oracle(p_out, n, report):
    from paper_2409_12892_amd import binding as B
    rng = np.random.default_rng(70 + p_out)
    par = bf16_params(p_out, 71)
    f = jacobian.round_bf16(rng.normal(size=(8, n)))
    t = rng.normal(size=(p_out, n)) * 0.5
    mask = rng.uniform(size=(p_out, n)) > 0.25
    loss_ref, g_ref = precond.loss_and_grad(par, f, t, mask)
    _, bar_s = forward_bar(par, f)
    bars = grad_bar(par, f, t, mask, bar_s)
    w = pack(par, p_out)
    tr = B.MlpTrainer(w.clone(), lr=1e-3)
    F = torch.from_numpy(f.astype(np.float32)).cuda()
    T = torch.from_numpy(t.astype(np.float32)).cuda()
    Mk = torch.from_numpy(mask.astype(np.float32)).cuda()
    loss, g = tr.step(F, T, Mk, lr=0.0, want_grad=True)
    assert tr.step_count == 0 and torch.equal(tr.w, w)         # lr = 0 leaves the weights alone
    g = unpack_grad(g, p_out)
    worst = 0.0
    for k in g_ref:
        err = np.abs(g[k] - g_ref[k])
        worst = max(worst, float(np.max(err / bars[k])))
        assert np.all(err <= bars[k]), (k, float(np.max(err / bars[k])))
    report[("mlp_grad", p_out, n)] = worst
    assert abs(loss.item() - loss_ref) <= 4 * U * loss_ref + 1e-9
    # one Adam step: from zero moments the step is lr g / (|g| + eps), i.e. -lr sign(g)
    # wherever the sign of the gradient is certain
    loss2, _ = tr.step(F, T, Mk)
    assert tr.step_count == 1 and abs(loss2.item() - loss.item()) == 0.0
    new = B.mlp_unpack(tr.w)
    old = B.mlp_unpack(w)
    m0 = {k: np.zeros_like(v) for k, v in g_ref.items()}
    ref_new = precond.adam_step(par, g_ref, m0, {k: np.zeros_like(v) for k, v in g_ref.items()}, 1, 1e-3)
    for k in g_ref:
        step = new[k] - old[k]
        if k in ("W3", "b3"):
            step = step[..., :p_out]
            assert np.all(new[k][..., p_out:] == old[k][..., p_out:])
        sure = (np.abs(g_ref[k]) > bars[k]) & (np.abs(g_ref[k]) > 1e-5)
        np.testing.assert_allclose(step[sure], (ref_new[k] - par[k])[sure], rtol=1e-3, atol=1e-9)
        assert np.all(np.abs(step) <= 1e-3 + 1e-6)


def test_mlp_empty_and_bad_arguments():
    from paper_2409_12892_amd import binding as B
    w = B.mlp_init(5)
    s, sc, nf = B.lm_mlp_forward(w, torch.zeros((8, 0), device="cuda"), 5)
    assert s.shape == (5, 0) and int(nf.item()) == 0
    tr = B.MlpTrainer(w)
    loss, g = tr.step(torch.zeros((8, 0), device="cuda"), torch.zeros((5, 0), device="cuda"),
                      torch.zeros((5, 0), device="cuda"), lr=0.0, want_grad=True)
    assert loss.item() == 0.0 and torch.count_nonzero(g).item() == 0
    with pytest.raises(RuntimeError):
        B.lm_mlp_forward(w, torch.zeros((8, 4), device="cuda"), 65)


# ---- training and use ---------------------------------------------------------------

def scene_data(B, seed, N=4000, views=(3, 96, 96)):
    p = make_problem("tiny", N=N, subsets=[views], seed=seed, deg=3, with_J=False)
    x = torch.from_numpy(p["scene"].x).cuda()
    tgt = torch.from_numpy(p["target"].ravel()).cuda()
    cache, b, _ = B.lm_build_cache(x, 3, p["cams"], tgt)
    M = B.lm_jacobi_diag(cache)
    feat = B.lm_precond_features(cache, x, M)
    t, mask = B.lm_precond_targets(cache, LAM, FLOOR)
    return dict(cache=cache, b=b, M=M, feat=feat, t=t, mask=mask)


def pcg_iters(B, d, scale):
    _, st = B.lm_pcg_solve([d["cache"]], [d["b"]], [d["M"]], LAM, 200, 1e-2, B.TOL_RELATIVE,
                           scales=None if scale is None else [scale], diag_floor=FLOOR)
    return st[0]["iters"]


def test_training_lowers_the_loss_and_the_learned_scale_cuts_pcg_iterations(report):
    """Trained on two SH-3 scenes, evaluated on a third: the loss falls, and
    on the held-out scene PCG with the learned scale needs fewer iterations
    than Jacobi to reach a relative residual of 1e-2, and at most a quarter
    more than the exact target scale (reported beside it)."""
    from paper_2409_12892_amd import binding as B
    print("[gpu precond] training scenes", flush=True)
    train = [scene_data(B, s) for s in (81, 82)]
    feat = torch.cat([d["feat"] for d in train], dim=1).contiguous()
    t = torch.cat([d["t"] for d in train], dim=1).contiguous()
    mask = torch.cat([d["mask"] for d in train], dim=1).contiguous()
    P = t.shape[0]
    tr = B.MlpTrainer(B.mlp_init(P, seed=3), lr=3e-3)
    first, _ = tr.step(feat, t, mask, lr=0.0)
    for _ in range(400):
        tr.step(feat, t, mask)
    last, _ = tr.step(feat, t, mask, lr=0.0)
    first, last = first.item(), last.item()
    print(f"[gpu precond] training loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.5 * first
    test = scene_data(B, 83)
    _, scale, nf = B.lm_mlp_forward(tr.w, test["feat"], P, want_s=False)
    assert int(nf.item()) == 0
    exact = torch.where(test["mask"] > 0, torch.exp(test["t"]), torch.ones_like(test["t"]))
    it_j = pcg_iters(B, test, None)
    it_l = pcg_iters(B, test, scale)
    it_t = pcg_iters(B, test, exact)
    report[("learned_precond_iters",)] = dict(jacobi=it_j, learned=it_l, exact_target=it_t, loss0=first, loss=last)
    print(f"[gpu precond] PCG iterations to 1e-2: jacobi {it_j}, learned {it_l}, exact target {it_t}", flush=True)
    assert it_l < it_j
    assert it_l <= 1.25 * it_t + 1
    for d in train + [test]:
        d["cache"].destroy()
