"""Explicit Jacobian of the rendered pixel colours with respect to every
Gaussian parameter, in float64, and the products the hot path computes.

Paper eq. backward-pass (section 3.3): dr/dx = dr/dc * dc/ds * ds/dx.  With
least-squares colour residuals r = c - C* (supplement A.4: dr/dc = 1 for L2),
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

Storing the cache in a 16-bit type (the low-precision cache of the hot
path) rounds each pair's T and dC/dalpha: T and D enter every Jacobian
entry linearly, J = D_ch * (dalpha/dy_geo . dy_geo/dx) + alpha T *
dc_ch/dx, so ``Jacobian.rounded(dtype)`` re-evaluates J with T and D
rounded as stored (float64 -> float32 -> bfloat16 or float16, round to
nearest even) and everything else exact.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .forward import project, render

_CSTEP = 1e-30


def round_bf16(v: np.ndarray) -> np.ndarray:
    """float64 -> float32 -> bfloat16 (round to nearest, ties to even),
    returned as float64."""
    f = np.ascontiguousarray(np.asarray(v, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(v: np.ndarray) -> np.ndarray:
    """float64 -> float32 -> IEEE binary16 (round to nearest even), returned
    as float64."""
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


CACHE_ROUNDING = {"f32": lambda v: np.asarray(v, np.float64).astype(np.float32).astype(np.float64),
                  "bf16": round_bf16, "f16": round_f16}


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


def dalpha_dygeo(pairs: dict, y: np.ndarray) -> np.ndarray:
    """Per-pair d alpha / d(m_x, m_y, A, B, C, o), zero for a clamped alpha."""
    a = pairs["alpha"]
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
    return np.stack([dadm_x, dadm_y, dadA, dadB, dadC, dado], axis=1)     # [n,6]


def dC_dy(pairs: dict, y: np.ndarray) -> np.ndarray:
    """Per-pair 3 x 9 block of d(pixel colour) / d(splat attributes)."""
    a = pairs["alpha"]
    T = pairs["T"]
    geo = dalpha_dygeo(pairs, y)
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
        rows, cols = [], []
        geo_part, col_part, Dn, Tn = [], [], [], []
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
                g = pairs["g"]
                n = len(g)
                # the pair's block dC/dy @ dy/dx, entry (ch, j) = D_ch * geo_j +
                # T * col_ch_j with geo = dalpha/dy_geo . dy_geo/dx_j and
                # col_ch = alpha dc_ch/dx_j (the two factors the cache stores
                # are kept apart)
                geo = dalpha_dygeo(pairs, pr["y"])                          # [n,6]
                gpart = np.einsum("nk,kjn->nj", geo, dydx[0:6][:, :, g])   # [n,P]
                cpart = pairs["alpha"][:, None, None] * np.transpose(dydx[6:9][:, :, g], (2, 0, 1))  # [n,3,P]
                r = roff + np.arange(3)[None, :, None] * (H * W) + pairs["pixel"][:, None, None]
                c = np.arange(self.P)[None, None, :] * self.N + g[:, None, None]
                rows.append(np.broadcast_to(r, (n, 3, self.P)).ravel())
                cols.append(np.broadcast_to(c, (n, 3, self.P)).ravel())
                geo_part.append(np.broadcast_to(gpart[:, None, :], (n, 3, self.P)).ravel())
                col_part.append(cpart.ravel())
                Dn.append(np.broadcast_to(pairs["D"][:, :, None], (n, 3, self.P)).ravel())
                Tn.append(np.broadcast_to(pairs["T"][:, None, None], (n, 3, self.P)).ravel())
            roff += 3 * H * W
        self.n_res = roff
        cat = (lambda lst: np.concatenate(lst)) if rows else (lambda lst: np.zeros(0))
        self._rows = cat(rows).astype(np.int64)
        self._cols = cat(cols).astype(np.int64)
        self._geo, self._col, self._D, self._T = cat(geo_part), cat(col_part), cat(Dn), cat(Tn)
        self._set_values(self._D * self._geo + self._T * self._col)

    def _set_values(self, vals: np.ndarray) -> None:
        # every (row, column) comes from one pair: a pixel meets a Gaussian once
        self.J = sp.csr_matrix((vals, (self._rows, self._cols)), shape=(self.n_res, self.P * self.N))
        self.J.sum_duplicates()
        self.JT = self.J.T.tocsr()

    def rounded(self, dtype: str) -> "Jacobian":
        """The Jacobian the products see when the cache stores T and
        dC/dalpha in `dtype` ("f32", "bf16" or "f16")."""
        out = object.__new__(Jacobian)
        out.__dict__.update(self.__dict__)
        rnd = CACHE_ROUNDING[dtype]
        out._set_values(rnd(self._D) * self._geo + rnd(self._T) * self._col)
        return out

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

    def apply_JtJ(self, p: np.ndarray, lam: float = 0.0, M: np.ndarray | None = None,
                  w: np.ndarray | None = None) -> np.ndarray:
        """J^T J p (+ lam M p).  With per-residual weights w (supplement A.4,
        eq. apply-jtj-simplified-vec-vec: w = (dr/dc)^2 of each pixel and
        channel) the product is J^T (w . J p), J being the colour Jacobian."""
        p = np.asarray(p, np.float64).ravel()
        u = self.apply_J(p)
        if w is not None:
            u = np.asarray(w, np.float64).ravel() * u
        g = self.apply_JT(u)
        if M is not None:
            g = g + lam * np.asarray(M, np.float64).ravel() * p
        return g

    def diag_JtJ(self, w: np.ndarray | None = None) -> np.ndarray:
        """diag(J^T J), or diag(J^T W J) = sum_i w_i J_ij^2 with weights."""
        sq = self.J.multiply(self.J)
        if w is None:
            return np.asarray(sq.sum(axis=0)).ravel()
        return np.asarray(sq.T @ np.asarray(w, np.float64).ravel()).ravel()

    def Jp_sqnorm(self, p: np.ndarray, w: np.ndarray | None = None) -> float:
        """||J p||^2, or sum_i w_i (J p)_i^2 with weights."""
        u = self.apply_J(p)
        return float(u @ u) if w is None else float(u @ (np.asarray(w, np.float64).ravel() * u))

    def weighted(self, w: np.ndarray) -> "Jacobian":
        """The Jacobian of the residuals r whose rows are sqrt(w_i) times the
        colour Jacobian's (eq. res-sq-root-weights with |dr/dc| = sqrt(w))."""
        out = object.__new__(Jacobian)
        out.__dict__.update(self.__dict__)
        s = np.sqrt(np.asarray(w, np.float64).ravel())
        out.J = sp.diags(s) @ self.J
        out.J = out.J.tocsr()
        out.JT = out.J.T.tocsr()
        return out

    def b(self, targets: list[np.ndarray]) -> np.ndarray:
        return -self.apply_JT(self.residual(targets))

    def JtJ(self) -> sp.csr_matrix:
        return (self.JT @ self.J).tocsr()

    @property
    def n_pairs(self) -> int:
        return int(sum(len(vw["raster"]["pairs"]["g"]) for vw in self.views))
