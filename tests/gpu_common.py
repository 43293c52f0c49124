"""Shared helpers for the GPU parity tests: seeded problems, oracle runs and
error metrics.  Inputs come from the scene generator; expected values come
from the oracle only."""
from __future__ import annotations

import numpy as np

from oracle import forward, jacobian, solve
from paper_2409_12892_amd import scenegen as sg

BLOCKS = {"mean": slice(0, 3), "scale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
          "sh": slice(11, None)}


def rel(a, b) -> float:
    """Norm-wise relative error ||a - b|| / ||b||."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def make_problem(name="tiny", N=None, subsets=None, seed=None, deg=None, tile=(16, 16), with_J=True):
    """Scene, cameras and targets (oracle render of the perturbed scene plus
    pixel noise, float32) for one subset, plus the oracle Jacobian at x."""
    d = sg.config_scene(name, N=N, subsets=subsets, seed=seed, deg=deg)
    sc = d["scene"]
    cams = d["cams"][0]
    tw, th = tile
    imgs = forward.render_images(d["x_star"], cams, sc.sh_degree, tw, th)
    target = np.stack([(im + nz).astype(np.float32) for im, nz in zip(imgs, d["noise"][0])])
    J = jacobian.Jacobian(sc.x, cams, sc.sh_degree, tw, th) if with_J else None
    return dict(scene=sc, cams=cams, target=target, J=J, cfg=d["cfg"], tile=tile)


def random_direction(P, N, seed, block=None):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 1.0, size=(P, N)).astype(np.float32)
    if block is not None:
        mask = np.zeros(P, bool)
        mask[BLOCKS[block]] = True
        p[~mask] = 0.0
    return p


def pcg_direction_bar(J, b, M, lam, n_iters, eps=1e-6, trials=3, diag_floor=0.0, tol=0.0, tol_mode=0,
                      precond=None, precond_eps=0.0):
    """Tolerance for a float32 PCG direction, derived from the problem's own
    sensitivity: the oracle reruns Algorithm 1 with every J^T J product
    perturbed element-wise by relative noise of size eps (the float32 budget
    of one product: ~10 accumulated roundings of 2^-24), and the bar is the
    largest change of the direction over the trials, never below 1e-4: a
    direction within it is indistinguishable from float32 product rounding.
    With a block preconditioner its output is perturbed by relative noise of
    size precond_eps as well (the float32 factorisation's error)."""
    base = solve.pcg(J.apply_JtJ, b, M, lam, n_iters, tol, tol_mode, diag_floor=diag_floor, precond=precond)["x"]
    worst = 0.0
    for t in range(trials):
        rng = np.random.default_rng(1000 + t)

        def A(v):
            y = J.apply_JtJ(v)
            return y * (1.0 + eps * rng.standard_normal(y.shape))

        pre = None
        if precond is not None:
            def pre(v):
                y = precond(v)
                return y * (1.0 + precond_eps * rng.standard_normal(y.shape))
        x = solve.pcg(A, b, M, lam, n_iters, tol, tol_mode, diag_floor=diag_floor, precond=pre)["x"]
        worst = max(worst, rel(x, base))
    return max(1e-4, worst)


def oracle_pcg(J, target, lam, n_iters, tol=0.0, tol_mode=0):
    b = J.b(list(target))
    M = J.diag_JtJ()
    out = solve.pcg(J.apply_JtJ, b, M, lam, n_iters, tol, tol_mode)
    return b, M, out


def kappa_max(blocks, lam, floor):
    """Largest condition number of the Jacobi-scaled damped blocks
    B_k + lam diag(max(d, floor)) over the observed parameters."""
    worst = 1.0
    for Bk in blocks:
        d = np.diag(Bk).copy()
        obs = d > 0
        if not obs.any():
            continue
        A = Bk[np.ix_(obs, obs)] + np.diag(lam * np.maximum(d[obs], floor))
        s = 1.0 / np.sqrt(np.diag(A))
        ev = np.linalg.eigvalsh(A * s[:, None] * s[None, :])
        worst = max(worst, ev.max() / ev.min())
    return worst
