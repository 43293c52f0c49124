"""Pins of the LM outer-step oracle (section 3.2, eq. line-search and
eq. tr-update): a scalar problem worked by hand, a linear least-squares
problem (where the Gauss-Newton model is exact, so rho = 1 and the grid line
search keeps the full step), the reject branch, and the algebraic identity
between the model decrease and b = -J^T F on a 3DGS scene."""
import math

import numpy as np
import pytest

from oracle import jacobian, lm, solve
from paper_2409_12892_amd import scenegen as sg


class _Dense:
    """apply_J / apply_JT / apply_JtJ / diag_JtJ of an explicit matrix."""

    def __init__(self, A):
        self.A = np.asarray(A, np.float64)

    def apply_J(self, p):
        return self.A @ np.asarray(p, np.float64).ravel()

    def apply_JT(self, u):
        return self.A.T @ np.asarray(u, np.float64).ravel()

    def apply_JtJ(self, p):
        return self.apply_JT(self.apply_J(p))

    def diag_JtJ(self):
        return (self.A * self.A).sum(axis=0)


def test_scalar_step_worked_by_hand():
    """F(x) = x^2 at x = 1, lambda = 1/2: J = 2, b = -2, M = 4, the damped
    system 6 delta = -2 gives delta = -1/3 (Algorithm 1 reaches it in one
    iteration); E(gamma) = (1 - gamma/3)^4 is smallest on the grid at
    gamma = 1, E1 = 16/81, the model value (J delta + F)^2 = 1/9, so
    rho = (1 - 16/81) / (1 - 1/9) = 65/72 and
    lambda_next = 1/2 (1 - (2 rho - 1)^3) = 1/2 (1 - (29/36)^3)."""
    res = lambda x: np.array([float(np.ravel(x)[0]) ** 2])
    out = lm.lm_step(np.array([1.0]), res, res, lambda x: _Dense([[2.0 * float(np.ravel(x)[0])]]), 0.5, 3,
                     lam_min=1e-9)
    assert out["delta"][0] == pytest.approx(-1.0 / 3.0, rel=1e-14)
    assert out["gamma"] == 1.0
    assert out["E1"] == pytest.approx(16.0 / 81.0, rel=1e-14)
    assert out["model"] == pytest.approx(1.0 / 9.0, rel=1e-14)
    assert out["rho"] == pytest.approx(65.0 / 72.0, rel=1e-13)
    assert out["accepted"]
    assert out["lam_next"] == pytest.approx(0.5 * (1.0 - (29.0 / 36.0) ** 3), rel=1e-13)
    np.testing.assert_allclose(out["x_next"], [2.0 / 3.0], rtol=1e-14)


def test_scalar_step_rejected_doubles_lambda_and_keeps_x():
    res = lambda x: np.array([float(np.ravel(x)[0]) ** 2])
    out = lm.lm_step(np.array([1.0]), res, res, lambda x: _Dense([[2.0 * float(np.ravel(x)[0])]]), 0.5, 3,
                     rho_min=0.95)
    assert not out["accepted"]
    assert out["lam_next"] == 1.0
    np.testing.assert_array_equal(out["x_next"], [1.0])


def test_linear_least_squares_gives_rho_one_and_the_full_step():
    """F(x) = A x - y: the model is exact, so rho = 1; the damped step's
    exact line minimiser gamma* = d^T b / ||A d||^2 is >= 1 (d^T b =
    d^T (A^T A + lambda D) d), so the grid keeps gamma = 1; lambda * (1 - 1)
    = 0 is clamped to lam_min.  With n_iters = dim Algorithm 1 is exact."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(40, 7))
    y = rng.normal(size=40)
    x0 = rng.normal(size=7)
    res = lambda x: A @ np.ravel(x) - y
    lam = 0.3
    out = lm.lm_step(x0, res, res, lambda x: _Dense(A), lam, 7, lam_min=1e-4)
    D = (A * A).sum(axis=0)
    ref = np.linalg.solve(A.T @ A + lam * np.diag(D), -A.T @ res(x0))
    np.testing.assert_allclose(out["delta"], ref, rtol=1e-9)
    assert out["gamma"] == 1.0
    assert out["rho"] == pytest.approx(1.0, abs=1e-10)
    assert out["lam_next"] == 1e-4
    d = out["delta"]
    assert d @ out["b"] >= np.sum((A @ d) ** 2)


def test_model_decrease_identity_on_a_scene():
    """On a 3DGS scene: ||F||^2 - ||J g d + F||^2 = 2 g d^T b - g^2 ||J d||^2
    (b = -J^T F), and an accepted step lowers the error."""
    d = sg.config_scene("tiny", N=300, subsets=[(2, 32, 32)], seed=21)
    sc, cams = d["scene"], d["cams"][0]
    from oracle import forward
    tg = [im + n for im, n in zip(forward.render_images(d["x_star"], cams, sc.sh_degree), d["noise"][0])]
    out = lm.lm_step_3dgs(sc.x, cams, tg, sc.sh_degree, 1e-2, 8, [0], diag_floor=1e-2)
    g, dl = out["gamma"], out["delta"].ravel()
    J = jacobian.Jacobian(sc.x, cams, sc.sh_degree)
    Jd = J.apply_J(dl)
    pred = 2 * g * float(dl @ out["b"]) - g * g * float(Jd @ Jd)
    assert out["E0"] - out["model"] == pytest.approx(pred, rel=1e-9)
    assert out["accepted"] and out["E1"] < out["E0"]
    assert out["E_ls"][out["k"]] == out["E_ls"].min()
