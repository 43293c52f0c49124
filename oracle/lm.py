"""One Levenberg-Marquardt outer step in float64 (paper section 3.2, "Apply
Parameter Update"): the damped normal equations solved by Algorithm 1, the
line search of eq. line-search and the trust-region ratio and damping update
of eq. tr-update.

Readings (the paper fixes the formulas, not these details):

* Line search: eq. line-search minimises E(x + gamma delta) over gamma on a
  30 % subset of the images; the method is not named.  Here the minimum is
  taken over a fixed grid of gammas (by default 1, 1/2, ..., 2^-12), every
  grid value evaluated on the line-search views, ties to the larger gamma.
* Ratio: rho = (||F(x)||^2 - ||F(x + g d)||^2) /
  (||F(x)||^2 - ||J g d + F(x)||^2), both norms over all images, the model
  norm taken with the explicit J.  A non-positive model decrease gives
  rho = -inf (the step is rejected).
* Update: keep the step when rho > rho_min (1e-5) and multiply lambda by
  1 - (2 rho - 1)^3; otherwise revert and double lambda.  For rho >= 1 the
  factor is <= 0, so the product leaves the admissible range; lambda is
  then clamped to [lam_min, lam_max] (the paper constrains lambda to such
  a range, section 4 "Implementation Details"), which is what keeps it
  positive.

The step is generic in the residual: ``residual(x)`` returns F(x) over all
images, ``residual_ls(x)`` over the line-search images, ``jacobian(x)``
returns an object with ``apply_J``, ``apply_JtJ`` and ``diag_JtJ`` (the
explicit Jacobian of ``oracle.jacobian`` for 3DGS).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import solve

GAMMAS = tuple(2.0 ** -k for k in range(13))


def lm_step(x, residual, residual_ls, jacobian, lam: float, n_iters: int, *, diag_floor: float = 0.0,
            gammas=GAMMAS, rho_min: float = 1e-5, lam_min: float = 1e-4, lam_max: float = 1e4,
            tol: float = 0.0, tol_mode: int = solve.TOL_NONE, J=None) -> dict:
    """One LM iteration from x (float64 [P][N] or a flat vector).

    Returns delta, the grid errors E_ls(gamma), gamma, E0 = ||F(x)||^2,
    E1 = ||F(x + gamma delta)||^2, the model value ||J gamma delta + F||^2,
    rho, whether the step is kept, lambda_next and the new x."""
    x = np.asarray(x, np.float64)
    J = jacobian(x) if J is None else J
    F = np.asarray(residual(x), np.float64).ravel()
    b = -np.asarray(J.apply_JT(F), np.float64).ravel()        # b = -J^T F (eq. norm-eq)
    M = np.asarray(J.diag_JtJ(), np.float64).ravel()
    out = solve.pcg(J.apply_JtJ, b, M, lam, n_iters, tol, tol_mode, diag_floor=diag_floor)
    delta = out["x"].reshape(x.shape)
    # eq. line-search on the grid, every value evaluated
    E_ls = np.array([float(np.sum(np.asarray(residual_ls(x + g * delta), np.float64) ** 2)) for g in gammas])
    k = int(np.flatnonzero(E_ls == E_ls.min())[0])
    gamma = float(gammas[k])
    x_new = x + gamma * delta
    F1 = np.asarray(residual(x_new), np.float64).ravel()
    E0 = float(F @ F)
    E1 = float(F1 @ F1)
    u = np.asarray(J.apply_J(gamma * delta.ravel()), np.float64).ravel() + F
    model = float(u @ u)
    denom = E0 - model
    rho = (E0 - E1) / denom if denom > 0 else -np.inf
    keep = bool(rho > rho_min and np.isfinite(E1))
    lam_next = lam * (1.0 - (2.0 * rho - 1.0) ** 3) if keep else 2.0 * lam
    lam_next = float(min(max(lam_next, lam_min), lam_max))
    return dict(delta=delta, b=b, M=M, pcg=out, E_ls=E_ls, k=k, gamma=gamma, E0=E0, E1=E1, model=model,
                rho=rho, accepted=keep, lam_next=lam_next, x_next=x_new if keep else x)


def lm_step_3dgs(x, cams, targets, deg: int, lam: float, n_iters: int, ls_views, TW: int = 16, TH: int = 16,
                 **kw) -> dict:
    """lm_step for the least-squares colour residuals F = render(x) - target
    of one image subset (section 3.1), the line search on the views listed
    in ls_views."""
    from .forward import render_images
    from .jacobian import Jacobian

    targets = [np.asarray(t, np.float64) for t in targets]
    ls_views = list(ls_views)
    ls_cams = cams.subset(ls_views)

    def residual(xx):
        return np.concatenate([(im - t).ravel() for im, t in zip(render_images(xx, cams, deg, TW, TH), targets)])

    def residual_ls(xx):
        imgs = render_images(xx, ls_cams, deg, TW, TH)
        return np.concatenate([(im - targets[v]).ravel() for im, v in zip(imgs, ls_views)])

    return lm_step(x, residual, residual_ls, lambda xx: Jacobian(xx, cams, deg, TW, TH), lam, n_iters, **kw)
