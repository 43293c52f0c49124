"""Levenberg-Marquardt outer loop around the HIP hot path (paper section 3.2).

One iteration: the gradient cache at x (b = -J^T F, ||F||^2), the Jacobi
diagonal M, Algorithm 1 for delta, the subset combination, then

* line search  min_gamma E(x + gamma delta) on a subset of the views
  (eq. line-search; the paper uses 30% of the images and does not name the
  method - here: gamma on the grid 1, 1/2, 1/4, ..., 2^-12, starting from the
  previous iteration's gamma; larger steps are tried while they lower the
  subset error, then smaller ones while they lower it or while no step has
  yet beaten E(x) on the subset, whose value comes from the cache's per-view
  residuals; the best evaluated gamma is taken);
* trust-region ratio (eq. tr-update)
      rho = (||F(x)||^2 - ||F(x + g d)||^2) / (||F(x)||^2 - ||J g d + F(x)||^2)
  with the model decrease 2 g d^T b - g^2 ||J d||^2; keep the step when
  rho > 1e-5 and scale lambda by 1 - (2 rho - 1)^3, otherwise revert and
  double lambda; lambda is clamped to [lam_min, lam_max].  ||F(x + g d)||^2
  comes from building the cache at the trial point, which is the next
  iteration's cache when the step is accepted (a rejected step rebuilds at
  x).

The solve uses a minimum LM diagonal (diag_floor, CERES's safeguard; the
paper follows CERES for the lambda schedule): on scenes with deeply occluded
Gaussians, diag(J^T J) reaches 1e-25 and plain Jacobi PCG returns steps of
order |F| / sqrt(diag) ~ 1e10 that no line search can rescue.

The objective is plain least squares (objective="l2") or the paper's
square-root L1 / SSIM residuals (objective="l1_ssim", eq. gn-loss): then the
cache's residual weights and b come from lm_cache_objective after every
build, every product is J^T W J, and the errors E compared by the line
search and the trust-region ratio are the objective's values.

Every product, render, reduction and vector update (d^T b through
lm_vec_dot, x + gamma delta through lm_vec_axpy) runs in the library; this
module only sequences calls and does the scalar bookkeeping of the line
search and the trust-region rule.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import binding as B


@dataclasses.dataclass
class LMConfig:
    lam: float = 1e-2
    lam_min: float = 1e-4
    lam_max: float = 1e4
    n_iters: int = 8
    tol: float = 0.0
    tol_mode: int = B.TOL_NONE
    rho_min: float = 1e-5
    # minimum LM diagonal (see lm_pcg_solve); 0 reproduces Algorithm 1 exactly
    diag_floor: float = 1e-2
    line_search_fraction: float = 0.3
    gammas: tuple = tuple(2.0 ** -k for k in range(13))
    tile: tuple = (16, 16)
    cache_dtype: str = "f32"
    objective: str = "l2"           # "l2" or "l1_ssim"
    precond: str = "jacobi"         # "jacobi" (Algorithm 1) or "block" (per-Gaussian block-Jacobi)
    obj_eps: float = B.OBJ_EPS
    thin_window: int = 0            # 0: full cache; K > 0: thinned cache (re-blend windows of K)


class LMSolver:
    """Holds the caches, workspaces and damping state of one problem
    (one image subset)."""

    def __init__(self, x, sh_degree: int, cams, target, cfg: LMConfig, ls_views=None):
        import torch
        self.x = x
        self.deg = sh_degree
        self.cams = cams
        self.target = target
        self.cfg = cfg
        self.lam = cfg.lam
        V = cams.V
        k = max(1, int(round(cfg.line_search_fraction * V)))
        self.ls_idx = np.asarray(ls_views if ls_views is not None else np.linspace(0, V - 1, k).round().astype(int))
        self.ls_cams = cams.subset(self.ls_idx)
        sizes = [3 * int(cams.W[v]) * int(cams.H[v]) for v in range(V)]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        self.ls_target = torch.cat([target[offs[v]:offs[v + 1]] for v in self.ls_idx]).contiguous()
        self.cache = None
        self.b = None
        self.fsq = None
        self.built_at_x = False
        self.k_prev = 0
        self.ws = None
        self.M = None
        self.delta = None
        self.comb = None
        self.x_try = torch.empty_like(x)
        self.history = []
        self.obj = None if cfg.objective == "l2" else B.objective(cfg.objective, eps=cfg.obj_eps)
        self.E_views = None

    def _E(self, x, cams, target) -> float:
        if self.obj is None:
            val, self.ws = B.lm_residual_sqnorm(x, self.deg, cams, target, tile=self.cfg.tile, workspace=self.ws)
        else:
            val, self.ws = B.lm_objective_value(x, self.deg, cams, target, self.obj, tile=self.cfg.tile,
                                                workspace=self.ws)
        return float(val.item())

    def _build(self, x):
        """Cache at x; self.fsq holds the objective's value there (device),
        self.E_views its per-view split (or None: taken from the cache)."""
        cfg = self.cfg
        self.E_views = None
        if self.obj is None:
            self.cache, self.b, self.fsq = B.lm_build_cache(x, self.deg, self.cams, self.target, tile=cfg.tile,
                                                            cache_dtype=cfg.cache_dtype, cache=self.cache, b=self.b,
                                                            thin_window=cfg.thin_window)
        else:
            # the build's own b = -J^T F belongs to the least-squares objective
            self.cache, _, _ = B.lm_build_cache(x, self.deg, self.cams, self.target, tile=cfg.tile,
                                                cache_dtype=cfg.cache_dtype, cache=self.cache, want_b=False,
                                                thin_window=cfg.thin_window)
            self.b, self.E_views = B.lm_cache_objective(self.cache, self.target, self.obj, b=self.b)
            self.fsq = self.E_views.sum().reshape(1)

    def iteration(self) -> dict:
        import torch
        cfg = self.cfg
        if not self.built_at_x:
            self._build(self.x)
        b, fsq = self.b, self.fsq
        self.M = B.lm_jacobi_diag(self.cache, out=self.M)
        deltas, stats = B.lm_pcg_solve([self.cache], [b], [self.M], self.lam, cfg.n_iters, cfg.tol, cfg.tol_mode,
                                       deltas=None if self.delta is None else [self.delta],
                                       diag_floor=cfg.diag_floor, block=cfg.precond == "block")
        self.delta = deltas[0]
        self.comb = B.lm_combine_subsets([self.delta], [self.M], out=self.comb)
        d = self.comb
        jd = B.lm_jp_sqnorm(self.cache, d)
        E0 = float(fsq.item())
        dTb = float(B.lm_vec_dot(d, b).item())
        Jd2 = float(jd.item())
        per_view = B.lm_cache_view_sqnorm(self.cache) if self.E_views is None else self.E_views
        E_ref = float(per_view[torch.as_tensor(self.ls_idx, device=per_view.device)].sum().item())
        # line search on the view subset (grid 2^-k, warm start at the last k)
        gammas = cfg.gammas
        evals = {}

        def E(k):
            if k not in evals:
                B.lm_vec_axpy(self.x, d, gammas[k], out=self.x_try)
                evals[k] = self._E(self.x_try, self.ls_cams, self.ls_target)
            return evals[k]

        k = min(self.k_prev, len(gammas) - 1)
        k0 = k
        while k > 0 and E(k - 1) < E(k):
            k -= 1
        if k == k0:
            while k + 1 < len(gammas) and (E(k + 1) < E(k) or min(evals.values()) >= E_ref):
                k += 1
        k = min(evals, key=lambda kk: (evals[kk], kk))
        self.k_prev = k
        g = gammas[k]
        B.lm_vec_axpy(self.x, d, g, out=self.x_try)
        # the cache at the trial point gives ||F(x + g d)||^2 and serves the
        # next iteration if the step is accepted
        self._build(self.x_try)
        E1 = float(self.fsq.item())
        pred = 2.0 * g * dTb - g * g * Jd2
        rho = (E0 - E1) / pred if pred > 0 else -np.inf
        accepted = bool(rho > cfg.rho_min and np.isfinite(E1))
        lam_old = self.lam
        if accepted:
            self.x.copy_(self.x_try)
            self.lam = self.lam * (1.0 - (2.0 * rho - 1.0) ** 3)
        else:
            self.lam = self.lam * 2.0
        self.built_at_x = accepted
        # for rho >= 1 the factor 1 - (2 rho - 1)^3 is <= 0: the clamp to
        # [lam_min, lam_max] (the paper's constrained range) keeps lambda positive
        self.lam = float(min(max(self.lam, cfg.lam_min), cfg.lam_max))
        rec = dict(E0=E0, E1=E1, gamma=g, rho=rho, accepted=accepted, lam=lam_old, lam_next=self.lam,
                   pcg_iters=stats[0]["iters"], pcg_rel_res_sq=float(stats[0]["history"][-1]),
                   line_search_evals=len(evals))
        self.history.append(rec)
        return rec

    def restart(self, x0, lam: float | None = None):
        """Start a new LM run from x0 (a device copy of the starting
        parameters) with the configured damping; the caches stay as
        workspaces and the first iteration builds at x0."""
        self.x.copy_(x0)
        self.lam = self.cfg.lam if lam is None else float(lam)
        self.built_at_x = False
        self.k_prev = 0

    def close(self):
        for h in (self.cache, self.ws):
            if h is not None:
                h.destroy()
