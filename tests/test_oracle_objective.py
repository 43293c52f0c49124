"""Pins of the oracle's square-root L1 / SSIM objective (eq. gn-loss,
supplement A.4) and of its weighted products, against closed forms, an
independent library routine, finite differences and brute force."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.ndimage

from oracle import forward, jacobian, objective as ob
from paper_2409_12892_amd import scenegen as sg

from test_oracle_pins import small_scene


def test_window_normalised_symmetric_centre():
    win = ob.gaussian_window()
    assert win.shape == (11, 11)
    assert win.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(win, win.T)
    np.testing.assert_array_equal(win, win[::-1, ::-1])
    k = np.arange(-5, 6)
    g0 = 1.0 / np.exp(-(k * k) / (2 * 1.5 ** 2)).sum()
    assert win[5, 5] == pytest.approx(g0 * g0, rel=1e-14)


def test_local_mean_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    img = rng.uniform(-0.2, 1.2, size=(13, 17))
    win = ob.gaussian_window()
    ref = scipy.ndimage.correlate(img, win, mode="constant", cval=0.0)
    np.testing.assert_allclose(ob.local_mean(img, win), ref, rtol=1e-13, atol=1e-15)


def test_identical_images_have_no_residual():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(3, 20, 23))
    t = ob.terms(x, x)
    assert np.all(t["ssim"] == 1.0)
    assert t["E"] == 0.0
    assert np.all(t["e"] == 0.0) and np.all(t["w"] == 0.0)


def test_constant_images_closed_form_interior_and_corner():
    a, b = 0.7, 0.3
    H = W = 30
    S, dS = ob.ssim_channel(np.full((H, W), a), np.full((H, W), b))
    # interior: window inside the image, means a and b, variances 0
    ref = (2 * a * b + ob.C1) / (a * a + b * b + ob.C1)
    np.testing.assert_allclose(S[5:-5, 5:-5], ref, rtol=1e-10)
    # corner: the in-image part of the window has weight s = (sum_{k>=0} g_k)^2,
    # so m_x = a s, s_xx = a^2 s (1 - s), s_xy = a b s (1 - s)
    k = np.arange(-5, 6)
    g = np.exp(-(k * k) / (2 * 1.5 ** 2))
    g /= g.sum()
    s = g[5:].sum() ** 2
    mx, my = a * s, b * s
    vx, vy, cxy = a * a * s * (1 - s), b * b * s * (1 - s), a * b * s * (1 - s)
    ref_c = ((2 * mx * my + ob.C1) * (2 * cxy + ob.C2)) / ((mx * mx + my * my + ob.C1) * (vx + vy + ob.C2))
    assert S[0, 0] == pytest.approx(ref_c, rel=1e-12)
    assert S[-1, -1] == pytest.approx(ref_c, rel=1e-12)


def test_ssim_centre_derivative_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(12, 14))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    S, dS = ob.ssim_channel(x, y)
    h = 1e-6
    for (i, j) in [(0, 0), (5, 6), (11, 13), (3, 12), (8, 1)]:
        xp = x.copy(); xp[i, j] += h
        xm = x.copy(); xm[i, j] -= h
        fd = (ob.ssim_channel(xp, y)[0][i, j] - ob.ssim_channel(xm, y)[0][i, j]) / (2 * h)
        assert dS[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9), (i, j)


def test_weight_is_sum_of_squared_residual_derivatives():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, size=(3, 10, 9))
    y = np.clip(x + rng.normal(0, 0.15, size=x.shape), 0, 1)
    t = ob.terms(x, y, eps=1e-12)
    h = 1e-7
    for (ch, i, j) in [(0, 0, 0), (1, 4, 4), (2, 9, 8), (0, 7, 2)]:
        xp = x.copy(); xp[ch, i, j] += h
        xm = x.copy(); xm[ch, i, j] -= h
        tp, tm = ob.terms(xp, y, eps=1e-12), ob.terms(xm, y, eps=1e-12)
        # r_t = sqrt(f_t) at this pixel as a function of its own colour
        dr1 = (np.sqrt(tp["f1"][ch, i, j]) - np.sqrt(tm["f1"][ch, i, j])) / (2 * h)
        dr2 = (np.sqrt(tp["f2"][ch, i, j]) - np.sqrt(tm["f2"][ch, i, j])) / (2 * h)
        assert t["w"][ch, i, j] == pytest.approx(dr1 * dr1 + dr2 * dr2, rel=1e-5)
        r1, r2 = np.sqrt(t["f1"][ch, i, j]), np.sqrt(t["f2"][ch, i, j])
        assert t["e"][ch, i, j] == pytest.approx(r1 * dr1 + r2 * dr2, rel=1e-5, abs=1e-12)


def test_weight_floor_and_l1_sign_at_zero():
    x = np.full((3, 12, 12), 0.5)
    y = x.copy()
    y[0, 6, 6] = 0.5 + 1e-9                # f1 = 0.8e-9 < eps
    t = ob.terms(x, y, eps=1e-4)
    d1 = ob.LAMBDA1
    assert t["w"][0, 6, 6] >= d1 * d1 / (4 * 1e-4) * (1 - 1e-12)
    assert np.isfinite(t["w"]).all()
    assert t["e"][1, 6, 6] == 0.0 and t["w"][1, 6, 6] == 0.0     # c == C: sign(0) = 0, SSIM = 1


def test_l2_kind_is_plain_least_squares():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, size=(3, 7, 5))
    y = rng.uniform(0, 1, size=(3, 7, 5))
    t = ob.terms(x, y, kind=ob.OBJ_L2)
    np.testing.assert_array_equal(t["e"], x - y)
    np.testing.assert_array_equal(t["w"], np.ones_like(x))
    assert t["E"] == pytest.approx(((x - y) ** 2).sum(), rel=1e-15)


def test_l1_gauss_newton_gradient_matches_objective_gradient():
    """With only the L1 term every residual depends on its own pixel, so
    2 J^T e is the exact gradient of E(x): finite differences of the
    rendered objective over the Gaussian parameters."""
    deg, N = 0, 10
    sc, rng = small_scene(N, deg, 11)
    cams = sg.fibonacci_cameras(1, 32, 32)
    x = sc.x.astype(np.float64)
    J = jacobian.Jacobian(x, cams, deg)
    img = J.images()[0]
    tgt = img + rng.normal(0, 0.05, size=img.shape)

    def E(xx):
        return ob.terms(forward.render_images(xx, cams, deg)[0], tgt, lam2=0.0)["E"]

    e = ob.terms(img, tgt, lam2=0.0)["e"].ravel()
    grad = 2.0 * J.apply_JT(e)
    sign0 = np.sign(img - tgt)
    checked = 0
    for j in range(x.shape[0]):
        for g in range(0, N, 3):
            h = 1e-7 * max(1.0, abs(x[j, g]))
            xp = x.copy(); xp[j, g] += h
            xm = x.copy(); xm[j, g] -= h
            ip = forward.render_images(xp, cams, deg)[0]
            im = forward.render_images(xm, cams, deg)[0]
            if not (np.array_equal(np.sign(ip - tgt), sign0) and np.array_equal(np.sign(im - tgt), sign0)):
                continue
            fd = (E(xp) - E(xm)) / (2 * h)
            assert grad[j * N + g] == pytest.approx(fd, rel=1e-5, abs=1e-7), (j, g)
            checked += 1
    assert checked > 0.7 * x.shape[0] * len(range(0, N, 3))


# ------------------------------------------------------------ weighted products
def _tiny():
    sc, rng = small_scene(30, 0, 12)
    cams = sg.fibonacci_cameras(2, 24, 24)
    J = jacobian.Jacobian(sc.x, cams, 0)
    w = rng.uniform(0.0, 3.0, size=J.n_res)
    p = rng.normal(size=J.P * J.N)
    return J, w, p


def test_unit_weights_reduce_to_plain_products():
    J, w, p = _tiny()
    one = np.ones(J.n_res)
    np.testing.assert_array_equal(J.apply_JtJ(p, w=one), J.apply_JtJ(p))
    np.testing.assert_allclose(J.diag_JtJ(one), J.diag_JtJ(), rtol=1e-14)
    assert J.Jp_sqnorm(p, one) == pytest.approx(J.Jp_sqnorm(p), rel=1e-15)


def test_weighted_products_equal_products_of_row_scaled_jacobian():
    J, w, p = _tiny()
    Jw = J.weighted(w)
    np.testing.assert_allclose(J.apply_JtJ(p, w=w), Jw.apply_JtJ(p), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(J.diag_JtJ(w), Jw.diag_JtJ(), rtol=1e-12, atol=1e-300)
    assert J.Jp_sqnorm(p, w) == pytest.approx(Jw.Jp_sqnorm(p), rel=1e-12)


def test_weighted_diag_brute_force_and_psd():
    J, w, p = _tiny()
    Jd = J.J.toarray()
    A = Jd.T @ (w[:, None] * Jd)
    np.testing.assert_allclose(np.diag(A), J.diag_JtJ(w), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(A @ p, J.apply_JtJ(p, w=w), rtol=1e-10, atol=1e-12 * np.abs(A @ p).max())
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= -1e-12 * ev.max()
