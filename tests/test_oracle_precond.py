"""Pins of the learned-preconditioner oracle (float64): GELU against the
normal CDF, the MLP gradient against central differences, targets against
closed forms, blocks against the dense Jacobian, feature invariances, and
the exact-target preconditioner against Jacobi."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import jacobian, precond, solve
from paper_2409_12892_amd import scenegen as sg


def test_gelu_is_x_times_normal_cdf_and_its_derivative():
    z = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(precond.gelu(z), z * scipy.special.ndtr(z), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (precond.gelu(z + h) - precond.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(precond.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    p_out, n = 7, 13
    params = precond.init_params(p_out, seed=3)
    for k in params:
        params[k] = params[k] + 0.1 * rng.normal(size=params[k].shape)
    f = rng.normal(size=(precond.N_FEAT, n))
    t = rng.normal(size=(p_out, n))
    mask = rng.uniform(size=(p_out, n)) > 0.3
    loss, g = precond.loss_and_grad(params, f, t, mask)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = precond.loss_and_grad(params, f, t, mask)
            flat[idx] = old - h
            lm, _ = precond.loss_and_grad(params, f, t, mask)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[name].reshape(-1)[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (name, idx)


def test_rowsum_scaling_closed_forms():
    lam = 0.1
    # diagonal block: row sum = (1 + lam) d_j  ->  t = -log(1 + lam)
    B = np.diag([2.0, 0.5, 3.0])[None]
    t, m = precond.rowsum_scaling(B, lam)
    np.testing.assert_allclose(t[:, 0], -math.log(1 + lam), rtol=1e-14)
    assert m.all()
    # 2 x 2 block [[a, b], [b, c]]
    a, b, c = 2.0, 0.7, 1.5
    t, m = precond.rowsum_scaling(np.array([[[a, b], [b, c]]]), lam)
    ref = [math.log(a / (a * (1 + lam) + b)), math.log(c / (c * (1 + lam) + b))]
    np.testing.assert_allclose(t[:, 0], ref, rtol=1e-13)
    # unobserved parameter: masked out, the rest as if it did not exist
    t, m = precond.rowsum_scaling(np.array([[[a, 0, b], [0, 0, 0], [b, 0, c]]]), lam)
    assert list(m[:, 0]) == [True, False, True]
    np.testing.assert_allclose(t[[0, 2], 0], ref, rtol=1e-13)
    # a negative coupling counts by its magnitude
    t, _ = precond.rowsum_scaling(np.array([[[a, -b], [-b, c]]]), lam)
    np.testing.assert_allclose(t[:, 0], ref, rtol=1e-13)
    # minimum diagonal: D = max(d, floor) in the damping and the reference
    floor = 1.0
    t, _ = precond.rowsum_scaling(np.diag([0.25, 4.0])[None], lam, diag_floor=floor)
    np.testing.assert_allclose(t[:, 0], [math.log(floor / (0.25 + lam * floor)), -math.log(1 + lam)], rtol=1e-14)


@pytest.fixture(scope="module")
def small():
    d = sg.config_scene("tiny", N=40, subsets=[(2, 32, 32)], seed=33, deg=1)
    sc = d["scene"]
    J = jacobian.Jacobian(sc.x, d["cams"][0], sc.sh_degree)
    return d, sc, J


def test_blocks_are_the_dense_jacobian_blocks(small):
    d, sc, J = small
    blocks = precond.gaussian_blocks(J)
    Jd = J.J.toarray()
    for k in (0, 7, 23):
        cols = [j * sc.N + k for j in range(sc.P)]
        np.testing.assert_allclose(blocks[k], Jd[:, cols].T @ Jd[:, cols], rtol=1e-12, atol=1e-300)
    diag = np.stack([np.diag(blocks[k]) for k in range(sc.N)], axis=1)
    np.testing.assert_allclose(diag.ravel(), J.diag_JtJ(), rtol=1e-12, atol=1e-300)


def test_features_are_scale_free(small):
    d, sc, J = small
    M = J.diag_JtJ().reshape(sc.P, sc.N)
    cov = np.bincount(np.concatenate([vw["raster"]["pairs"]["g"] for vw in J.views]), minlength=sc.N)
    f = precond.features(M, cov, sc.x)
    f2 = precond.features(10.0 * M, 3 * cov, sc.x)
    np.testing.assert_allclose(f2[0:5], f[0:5], atol=1e-12)
    obs = M.sum(axis=0) > 0
    assert np.all(f[:, ~obs] == 0)
    x64 = sc.x.astype(np.float64)
    np.testing.assert_allclose(f[6][obs], 1 / (1 + np.exp(-x64[10][obs])), rtol=1e-15)
    np.testing.assert_allclose(f[7][obs], x64[3:6, obs].mean(axis=0), rtol=1e-15)


def test_exact_target_preconditioner_beats_jacobi():
    """On an SH-degree-3 scene the exact (shrunk) row-sum scaling needs fewer
    PCG iterations than Jacobi to reach a 1e-2 relative residual."""
    from oracle import forward
    d = sg.config_scene("tiny", N=300, subsets=[(2, 48, 48)], seed=34, deg=3)
    sc = d["scene"]
    J = jacobian.Jacobian(sc.x, d["cams"][0], sc.sh_degree)
    lam, floor = 1e-2, 1e-2
    target = [im + n for im, n in zip(forward.render_images(d["x_star"], d["cams"][0], 3), d["noise"][0])]
    b = J.b(target)
    M = J.diag_JtJ()
    t, mask = precond.targets(precond.gaussian_blocks(J), lam, diag_floor=floor)
    scale = np.where(mask, np.exp(t), 1.0).ravel()
    it_j = solve.pcg(J.apply_JtJ, b, M, lam, 200, 1e-2, solve.TOL_RELATIVE, diag_floor=floor)["iters"]
    it_t = solve.pcg(J.apply_JtJ, b, M, lam, 200, 1e-2, solve.TOL_RELATIVE, precond_scale=scale,
                     diag_floor=floor)["iters"]
    assert it_t < it_j


def test_adam_moves_by_lr_times_sign_under_a_constant_gradient():
    """With bias correction, a constant gradient g gives m_hat = g and
    v_hat = g^2 at every step, so each step moves by lr g / (|g| + eps)."""
    params = {"a": np.array([1.0, -2.0, 0.5, 3.0])}
    g = {"a": np.array([0.3, -4.0, 1e-3, -2e-2])}
    m = {"a": np.zeros(4)}
    v = {"a": np.zeros(4)}
    lr = 1e-2
    p = params
    for step in range(1, 6):
        new = precond.adam_step(p, g, m, v, step, lr)
        np.testing.assert_allclose(new["a"] - p["a"], -lr * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-9)
        p = new


def test_shrinkage_keeps_the_mean_and_scales_the_spread():
    rng = np.random.default_rng(9)
    t = rng.normal(size=(4, 50))
    mask = rng.uniform(size=(4, 50)) > 0.3
    mask[2] = False
    for beta in (0.0, 0.5, 1.0):
        s = precond.shrink_to_mean(t, mask, beta)
        assert np.all(s[~mask] == 0)
        for j in (0, 1, 3):
            o = mask[j]
            assert abs(s[j][o].mean() - t[j][o].mean()) < 1e-12
            np.testing.assert_allclose(s[j][o] - s[j][o].mean(), beta * (t[j][o] - t[j][o].mean()), atol=1e-12)
    np.testing.assert_allclose(precond.shrink_to_mean(t, mask, 1.0)[mask], t[mask], rtol=0, atol=1e-15)
    # the default target is the row-sum scaling shrunk by one half
    B = np.stack([np.diag([2.0, 0.5]), np.array([[2.0, 0.7], [0.7, 1.5]])])
    raw, m = precond.rowsum_scaling(B, 0.1)
    sh, m2 = precond.targets(B, 0.1)
    np.testing.assert_array_equal(m, m2)
    np.testing.assert_allclose(sh, precond.shrink_to_mean(raw, m, 0.5), rtol=1e-15)



def _parameter_groups_from_the_projection(deg=1):
    """Name the parameter rows by what they change in the projected splat
    (section 3.1 forward model), independently of any slice table: the
    mean rows move the 2D mean; the covariance rows change the conic but not
    the mean, and among them the quaternion rows are the ones whose radial
    direction changes nothing (the quaternion is normalised); the opacity
    row changes only the opacity; the SH rows change only the colour."""
    from oracle import forward
    d = sg.config_scene("tiny", N=6, subsets=[(1, 32, 32)], seed=41, deg=deg)
    cam = d["cams"][0].view(0)
    x = d["scene"].x.astype(np.float64)
    P = x.shape[0]
    base = forward.project(x, cam, deg)["y"]
    moved = {}
    for j in range(P):
        xc = x.astype(np.complex128)
        xc[j] += 1e-30j
        dy = np.abs(np.imag(forward.project(xc, cam, deg)["y"])) / 1e-30
        moved[j] = dict(mean=dy[0:2].max() > 0, conic=dy[2:5].max() > 0, opac=dy[5].max() > 0,
                        colour=dy[6:9].max() > 0, size=dy.max())
    mean_rows = [j for j in range(P) if moved[j]["mean"]]
    cov_rows = [j for j in range(P) if moved[j]["conic"] and not moved[j]["mean"]]
    # radial direction of the quaternion: x[q] += eps x[q] leaves y unchanged
    # (zero up to rounding: below 1e-9 of the rows' own derivatives)
    quat_rows = []
    for a in range(len(cov_rows) - 3):
        rows = cov_rows[a:a + 4]
        xc = x.astype(np.complex128)
        xc[rows] += 1e-30j * x[rows]
        radial = np.abs(np.imag(forward.project(xc, cam, deg)["y"])).max() / 1e-30
        if radial < 1e-9 * max(moved[j]["size"] for j in rows):
            quat_rows = rows
    scale_rows = [j for j in cov_rows if j not in quat_rows]
    opac_rows = [j for j in range(P) if moved[j]["opac"] and not moved[j]["conic"] and not moved[j]["mean"]]
    sh_rows = [j for j in range(P) if moved[j]["colour"] and not (moved[j]["conic"] or moved[j]["opac"])
               and not moved[j]["mean"]]
    assert np.all(base[5] > 0)
    return dict(mean=mean_rows, scale=scale_rows, quat=quat_rows, opacity=opac_rows, sh=sh_rows)


def test_feature_groups_follow_the_parameters_they_name():
    """Features 0-4 average the Jacobi diagonal over the mean, log-scale,
    quaternion, opacity and SH rows, identified here by their effect on the
    projection; computed per Gaussian with explicit loops over those rows."""
    groups = _parameter_groups_from_the_projection(deg=1)
    P = 11 + 3 * 4
    assert sorted(sum(groups.values(), [])) == list(range(P))
    assert [len(groups[k]) for k in ("mean", "scale", "quat", "opacity", "sh")] == [3, 3, 4, 1, 12]
    for i, k in enumerate(("mean", "scale", "quat", "opacity", "sh")):
        a, b = precond.GROUPS[i]
        assert list(range(P)[a:b]) == groups[k], k
    rng = np.random.default_rng(7)
    N = 9
    M = np.exp(rng.normal(0.0, 2.0, size=(P, N)))
    M[:, 4] = 0.0                                   # an unobserved Gaussian
    cov = rng.integers(1, 50, size=N).astype(np.float64)
    x = rng.normal(size=(P, N))
    f = precond.features(M, cov, x)
    obs = [k for k in range(N) if M[:, k].sum() > 0]
    for i, name in enumerate(("mean", "scale", "quat", "opacity", "sh")):
        raw = {}
        for k in obs:
            tot = 0.0
            for j in groups[name]:
                tot += M[j, k]
            raw[k] = math.log(tot / len(groups[name]))
        ref = sum(raw.values()) / len(obs)
        for k in obs:
            assert f[i, k] == pytest.approx(raw[k] - ref, abs=1e-12), (name, k)
        assert f[i, 4] == 0.0
    raw5 = {k: math.log(1.0 + cov[k]) for k in obs}
    ref5 = sum(raw5.values()) / len(obs)
    for k in obs:
        assert f[5, k] == pytest.approx(raw5[k] - ref5, abs=1e-12)
        assert f[6, k] == pytest.approx(1.0 / (1.0 + math.exp(-x[groups["opacity"][0], k])), rel=1e-14)
        assert f[7, k] == pytest.approx(sum(x[j, k] for j in groups["scale"]) / 3.0, rel=1e-13)
