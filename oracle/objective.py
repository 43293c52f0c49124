"""Residuals of the paper's rendering objective and their colour-space
derivatives, in float64.

Section 3.1 (eq. sgd-loss, eq. gn-loss): per pixel i and colour channel the
objective has two residuals, the square roots of an L1 term and of an SSIM
term,

    f1 = lam1 |c - C|,   f2 = lam2 (1 - SSIM(c, C)),   r_t = sqrt(f_t),

with lam1 = 0.8 and lam2 = 0.2, and E = sum over pixels and channels of
r1^2 + r2^2 = f1 + f2.  Supplement A.4 (eq. res-sq-root-weights,
res-sq-root-weights-sum, apply-jtj-simplified-vec-vec) factors every
Jacobian row into dr/dc (a per-pixel scalar) times dc/dx (the colour
Jacobian of the cache), so a Gauss-Newton step needs two per-pixel images:

    e = sum_t r_t dr_t/dc         (then b = -J_c^T e)
    w = sum_t (dr_t/dc)^2         (then J^T J p = J_c^T (w . J_c p)).

With r = sqrt(f):  r dr/dc = f'/2 exactly, and (dr/dc)^2 = f'^2 / (4 f).

SSIM (section 3.3: the SSIM residual's derivative goes to the centre pixel
only) follows its standard definition per colour channel: Gaussian-weighted
local means, variances and covariance over an 11 x 11 window of standard
deviation 1.5 (normalised to sum 1), with C1 = (0.01 L)^2, C2 = (0.03 L)^2 for
the dynamic range L = 1; pixels outside the image count as 0 in both images.

Readings where the paper is silent:
* the weight is singular where a residual vanishes (f' / sqrt f); the
  denominator takes max(f_t, eps) (eps a parameter), e stays exact;
* sign(0) = 0 for the L1 derivative;
* f2 is clamped at 0 (rounding can put SSIM a hair above 1).

For the plain least-squares objective (the default of the hot path,
LM_OBJ_L2) r = c - C: e = r, w = 1, E = sum r^2.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

LAMBDA1 = 0.8
LAMBDA2 = 0.2
WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
EPS = 1e-4

OBJ_L2 = 0
OBJ_L1_SSIM = 1


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """2-D window: the outer product of a sampled 1-D Gaussian normalised
    to sum 1."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    g = g / g.sum()
    return np.outer(g, g)


def local_mean(img: np.ndarray, win: np.ndarray) -> np.ndarray:
    """sum_{a,b} win[a,b] img[y + a - r, x + b - r], img zero outside."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    r = win.shape[0] // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for a in range(win.shape[0]):
        for b in range(win.shape[1]):
            out += win[a, b] * pad[a:a + H, b:b + W]
    return out


def ssim_channel(x: np.ndarray, y: np.ndarray, win: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """SSIM map of one channel and its derivative with respect to the
    centre pixel of each window (the other pixels' influence ignored)."""
    win = gaussian_window() if win is None else win
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g0 = win[win.shape[0] // 2, win.shape[1] // 2]
    mx, my = local_mean(x, win), local_mean(y, win)
    sxx = local_mean(x * x, win) - mx * mx
    syy = local_mean(y * y, win) - my * my
    sxy = local_mean(x * y, win) - mx * my
    A = 2.0 * mx * my + C1
    B = 2.0 * sxy + C2
    Cc = mx * mx + my * my + C1
    D = sxx + syy + C2
    S = (A * B) / (Cc * D)
    # d/dx_centre of mx, sxx, sxy: g0, 2 g0 (x - mx), g0 (y - my)
    dA = 2.0 * g0 * my
    dB = 2.0 * g0 * (y - my)
    dCc = 2.0 * g0 * mx
    dD = 2.0 * g0 * (x - mx)
    dS = (dA * B + A * dB) / (Cc * D) - S * (dCc * D + Cc * dD) / (Cc * D)
    return S, dS


def terms(image: np.ndarray, target: np.ndarray, kind: int = OBJ_L1_SSIM, lam1: float = LAMBDA1,
          lam2: float = LAMBDA2, eps: float = EPS) -> dict:
    """Residual terms of one view, image and target [3][H][W].

    Returns E (float), e and w ([3][H][W]) and, for the L1/SSIM objective,
    the per-term f1, f2 and derivatives d1 = f1', d2 = f2'."""
    c = np.asarray(image, np.float64)
    t = np.asarray(target, np.float64)
    if kind == OBJ_L2:
        r = c - t
        return dict(E=float((r * r).sum()), e=r, w=np.ones_like(r))
    diff = c - t
    f1 = lam1 * np.abs(diff)
    d1 = lam1 * np.sign(diff)
    S = np.empty_like(c)
    dS = np.empty_like(c)
    for ch in range(c.shape[0]):
        S[ch], dS[ch] = ssim_channel(c[ch], t[ch])
    f2 = np.maximum(lam2 * (1.0 - S), 0.0)
    d2 = -lam2 * dS
    e = 0.5 * (d1 + d2)
    w = d1 * d1 / (4.0 * np.maximum(f1, eps)) + d2 * d2 / (4.0 * np.maximum(f2, eps))
    return dict(E=float(f1.sum() + f2.sum()), e=e, w=w, f1=f1, f2=f2, d1=d1, d2=d2, ssim=S)


def terms_views(images: list, targets: list, kind: int = OBJ_L1_SSIM, lam1: float = LAMBDA1,
                lam2: float = LAMBDA2, eps: float = EPS) -> dict:
    """terms() of every view, e and w flattened in residual order
    [view][channel][row][col], E summed."""
    out = [terms(im, tg, kind, lam1, lam2, eps) for im, tg in zip(images, targets)]
    return dict(E=float(sum(o["E"] for o in out)),
                e=np.concatenate([o["e"].ravel() for o in out]),
                w=np.concatenate([o["w"].ravel() for o in out]))
