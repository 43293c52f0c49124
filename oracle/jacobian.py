"""Explicit Jacobian of the rendered pixel colours with respect to every
Gaussian parameter, in float64, and the products the hot path computes.

Paper eq. backward-pass (section 3.3): dr/dx = dr/dc * dc/ds * ds/dx.  With
least-squares colour residuals r = c - C* (supplement A.5: dr/dc = 1 for L2),
each contributing (pixel, splat) pair owns a dense 3 x P block

    J_pair = dC/dy (3 x 9)  @  dy/dx (9 x P)

where y = (m_x, m_y, A, B, C, o, r, g, b) is the projected splat.

* dC/dy follows from eq. alpha-blending with the active set frozen:
  dC_ch/dalpha = T c_ch - S_ch / (1 - alpha) (S = later contributions),
  dC_ch/dc_ch = alpha T, and alpha = o exp(power) gives
  dalpha/dm = alpha (A dx + B dy, B dx + C dy),
  dalpha/d(A,B,C) = alpha (-dx^2/2, -dx dy, -dy^2/2), dalpha/do = exp(power);
  a clamped alpha (0.99) has zero derivative.
* dy/dx is taken by complex-step differentiation of the float64 projection
  (exact to rounding; no truncation error), one step per parameter row.

The assembled J is a SciPy CSR matrix with rows indexed like the residual
images [view][channel][row][col] and columns like the structure-of-arrays
parameter vector x[P][N] flattened (j * N + g).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .forward import project, render

_CSTEP = 1e-30


def dydx_complex_step(x: np.ndarray, cam: dict, deg: int) -> np.ndarray:
    """d y / d x for every Gaussian in one view: array [9, P, N]."""
    x64 = np.asarray(x, dtype=np.float64)
    P, N = x64.shape
    out = np.zeros((9, P, N))
    for j in range(P):
        xc = x64.astype(np.complex128)
        xc[j] += 1j * _CSTEP
        yc = project(xc, cam, deg)["y"]
        out[:, j, :] = np.imag(yc) / _CSTEP
    return out


def dC_dy(pairs: dict, y: np.ndarray) -> np.ndarray:
    """Per-pair 3 x 9 block of d(pixel colour) / d(splat attributes)."""
    a = pairs["alpha"]
    T = pairs["T"]
    G = pairs["G"]
    dx = pairs["dx"]
    dy = pairs["dy"]
    g = pairs["g"]
    A, B, C = (np.real(y[i])[g] for i in (2, 3, 4))
    live = ~pairs["clamped"]
    dadm_x = np.where(live, a * (A * dx + B * dy), 0.0)
    dadm_y = np.where(live, a * (B * dx + C * dy), 0.0)
    dadA = np.where(live, -0.5 * a * dx * dx, 0.0)
    dadB = np.where(live, -a * dx * dy, 0.0)
    dadC = np.where(live, -0.5 * a * dy * dy, 0.0)
    dado = np.where(live, G, 0.0)
    geo = np.stack([dadm_x, dadm_y, dadA, dadB, dadC, dado], axis=1)        # [n,6]
    out = np.zeros((len(a), 3, 9))
    out[:, :, 0:6] = pairs["D"][:, :, None] * geo[:, None, :]
    for ch in range(3):
        out[:, ch, 6 + ch] = a * T
    return out


class Jacobian:
    """Explicit J for a set of views rendered from x (float64)."""

    def __init__(self, x: np.ndarray, cams, deg: int, TW: int = 16, TH: int = 16,
                 views: list[dict] | None = None):
        x64 = np.asarray(x, dtype=np.float64)
        self.P, self.N = x64.shape
        self.deg = deg
        self.views = render(x64, cams, deg, TW, TH) if views is None else views
        rows, cols, vals = [], [], []
        roff = 0
        self.row_offsets = []
        for vw in self.views:
            cam = vw["cam"]
            W, H = cam["W"], cam["H"]
            pr = vw["proj"]
            pairs = vw["raster"]["pairs"]
            self.row_offsets.append(roff)
            if len(pairs["g"]):
                dydx = dydx_complex_step(x64, cam, deg)                     # [9,P,N]
                dcdy = dC_dy(pairs, pr["y"])                                # [n,3,9]
                g = pairs["g"]
                blk = np.einsum("nci,ijn->ncj", dcdy, dydx[:, :, g])        # [n,3,P]
                n = len(g)
                r = roff + np.arange(3)[None, :, None] * (H * W) + pairs["pixel"][:, None, None]
                c = np.arange(self.P)[None, None, :] * self.N + g[:, None, None]
                rows.append(np.broadcast_to(r, (n, 3, self.P)).ravel())
                cols.append(np.broadcast_to(c, (n, 3, self.P)).ravel())
                vals.append(blk.ravel())
            roff += 3 * H * W
        self.n_res = roff
        if rows:
            rows = np.concatenate(rows)
            cols = np.concatenate(cols)
            vals = np.concatenate(vals)
        else:
            rows = cols = np.zeros(0, dtype=np.int64)
            vals = np.zeros(0)
        self.J = sp.csr_matrix((vals, (rows, cols)), shape=(self.n_res, self.P * self.N))
        self.J.sum_duplicates()
        self.JT = self.J.T.tocsr()

    # ---- images and residuals ----
    def images(self) -> list[np.ndarray]:
        return [vw["raster"]["image"] for vw in self.views]

    def residual(self, targets: list[np.ndarray]) -> np.ndarray:
        """F = rendered - target for every pixel and channel (L2 residuals)."""
        return np.concatenate([(vw["raster"]["image"] - np.asarray(t, np.float64)).ravel()
                               for vw, t in zip(self.views, targets)])

    # ---- products (eq. apply-j, apply-jt, diag-jtj) ----
    def apply_J(self, p: np.ndarray) -> np.ndarray:
        return self.J @ np.asarray(p, np.float64).ravel()

    def apply_JT(self, u: np.ndarray) -> np.ndarray:
        return self.JT @ np.asarray(u, np.float64).ravel()

    def apply_JtJ(self, p: np.ndarray, lam: float = 0.0, M: np.ndarray | None = None) -> np.ndarray:
        p = np.asarray(p, np.float64).ravel()
        g = self.apply_JT(self.apply_J(p))
        if M is not None:
            g = g + lam * np.asarray(M, np.float64).ravel() * p
        return g

    def diag_JtJ(self) -> np.ndarray:
        return np.asarray(self.J.multiply(self.J).sum(axis=0)).ravel()

    def b(self, targets: list[np.ndarray]) -> np.ndarray:
        return -self.apply_JT(self.residual(targets))

    def JtJ(self) -> sp.csr_matrix:
        return (self.JT @ self.J).tocsr()

    @property
    def n_pairs(self) -> int:
        return int(sum(len(vw["raster"]["pairs"]["g"]) for vw in self.views))
