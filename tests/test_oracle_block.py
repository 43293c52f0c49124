"""Pins of the oracle's block-Jacobi preconditioner (per-Gaussian damped
blocks of eq. norm-eq, inverted exactly)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import jacobian, precond, solve
from paper_2409_12892_amd import scenegen as sg

from test_oracle_pins import _disjoint_colour_problem, small_scene


def test_block_diagonal_system_is_solved_by_the_first_iterate():
    """Gaussians that never share a pixel make J^T J block-diagonal by
    Gaussian, so x0 = A^-1 b is already the damped normal-equation solution."""
    x, cams = _disjoint_colour_problem(deg=1)
    J = jacobian.Jacobian(x, cams, 1)
    JtJ = J.JtJ().toarray()
    N = J.N
    owner = np.arange(J.P * N) % N
    assert np.abs(JtJ[owner[:, None] != owner[None, :]]).max() == 0.0
    rng = np.random.default_rng(3)
    targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
    b = J.b(targets)
    M = J.diag_JtJ()
    for lam, floor in [(0.3, 0.0), (1e-2, 1e-2)]:
        pre = solve.block_jacobi(precond.gaussian_blocks(J), lam, floor)
        out = solve.pcg(J.apply_JtJ, b, M, lam, 0, diag_floor=floor, precond=pre)
        ref = solve.dense_solve(JtJ, b, lam, floor)
        np.testing.assert_allclose(out["x"], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_blocks_inverted_against_dense_submatrices():
    sc, rng = small_scene(20, 0, 17)
    cams = sg.fibonacci_cameras(2, 32, 32)
    J = jacobian.Jacobian(sc.x, cams, 0)
    P, N = J.P, J.N
    lam, floor = 0.05, 1e-2
    pre = solve.block_jacobi(precond.gaussian_blocks(J), lam, floor)
    v = rng.normal(size=P * N)
    z = pre(v).reshape(P, N)
    A = J.JtJ().toarray()
    V = v.reshape(P, N)
    for k in range(N):
        idx = np.arange(P) * N + k
        Ak = A[np.ix_(idx, idx)]
        d = np.diag(Ak).copy()
        obs = d > 0
        Ak = Ak + np.diag(lam * np.maximum(d, floor))
        np.testing.assert_allclose(Ak[np.ix_(obs, obs)] @ z[obs, k], V[obs, k], rtol=1e-9,
                                   atol=1e-12 * np.abs(V[:, k]).max())
        np.testing.assert_array_equal(z[~obs, k], V[~obs, k])


def test_block_jacobi_pcg_converges_to_dense_solve():
    sc, rng = small_scene(25, 1, 18)
    cams = sg.fibonacci_cameras(2, 32, 32)
    J = jacobian.Jacobian(sc.x, cams, 1)
    targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
    b = J.b(targets)
    M = J.diag_JtJ()
    lam = 0.1
    pre = solve.block_jacobi(precond.gaussian_blocks(J), lam)
    out = solve.pcg(J.apply_JtJ, b, M, lam, 400, tol=1e-24, tol_mode=solve.TOL_PAPER_SQUARED, precond=pre)
    ref = solve.dense_solve(J.JtJ(), b, lam)
    assert np.linalg.norm(out["x"] - ref) <= 1e-6 * np.linalg.norm(ref)
    # and it needs fewer iterations than Jacobi to a relative residual of 1e-2
    it_b = solve.pcg(J.apply_JtJ, b, M, lam, 200, tol=1e-4, tol_mode=solve.TOL_PAPER_SQUARED, precond=pre)["iters"]
    it_j = solve.pcg(J.apply_JtJ, b, M, lam, 200, tol=1e-4, tol_mode=solve.TOL_PAPER_SQUARED)["iters"]
    assert it_b < it_j
