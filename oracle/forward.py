"""Forward model of 3DGS in float64: projection, tile binning, alpha-blending.

Paper section 3.1 reviews the model and defers its details to the original
3DGS rasteriser; the conventions used here are the readings listed in the
design notes (pixel centres at +0.5, 0.3 px^2 dilation, 3-sigma radius,
alpha clamp 0.99, alpha threshold 1/255, transmittance cut-off 1e-4, near
plane 0.2, black background, colour offset 0.5 clamped at 0).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

from .sh import sh_basis

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
NEAR = 0.2
DILATION = 0.3


def _cam64(cam: dict):
    R = np.asarray(cam["R"], dtype=np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    return R, t, float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix [3,3,...] of the normalised quaternion q = (w,x,y,z)."""
    n = np.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
    w, x, y, z = q[0] / n, q[1] / n, q[2] / n, q[3] / n
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def project(x: np.ndarray, cam: dict, deg: int) -> dict:
    """Project every Gaussian into one view (paper section 3.1, EWA splatting
    of the original rasteriser).

    x: [P, N] float64 or complex128 (complex for complex-step derivatives).
    Returns y = [9, N] (m_x, m_y, conic A, B, C, opacity, r, g, b) plus the
    depth z, integer radius, visibility and per-channel colour-clamp flags.
    The conic (A, B, C) is the inverse 2D covariance [[A, B], [B, C]], so the
    Gaussian's exponent at offset d is -0.5*(A dx^2 + C dy^2) - B dx dy.
    """
    Rv, tv, fx, fy, cx, cy = _cam64(cam)
    K = (deg + 1) ** 2
    N = x.shape[1]
    mu = x[0:3]
    tc = Rv @ mu + tv[:, None]
    tx, ty, tz = tc[0], tc[1], tc[2]

    Rq = quat_to_rot(x[6:10])                               # [3,3,N]
    s2 = np.exp(2.0 * x[3:6])                               # [3,N]
    sigma = np.einsum("ikn,kn,jkn->ijn", Rq, s2, Rq)        # R diag(e^2s) R^T
    wcam = np.einsum("ai,ijn,bj->abn", Rv, sigma, Rv)       # camera frame

    zero = np.zeros_like(tz)
    Jp = np.array([[fx / tz, zero, -fx * tx / (tz * tz)],
                   [zero, fy / tz, -fy * ty / (tz * tz)]])  # [2,3,N]
    cov = np.einsum("ain,ijn,bjn->abn", Jp, wcam, Jp)
    a = cov[0, 0] + DILATION
    b = cov[0, 1]
    c = cov[1, 1] + DILATION
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det

    mx = fx * tx / tz + cx
    my = fy * ty / tz + cy
    opac = 1.0 / (1.0 + np.exp(-x[10]))

    cpos = -Rv.T @ tv
    dvec = mu - cpos[:, None]
    dn = np.sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2])
    dirs = dvec / dn
    Y = sh_basis(dirs, deg)                                 # [K,N]
    f = x[11:11 + 3 * K].reshape(K, 3, N)
    raw = 0.5 + np.einsum("kn,kcn->cn", Y, f)
    clamp = np.real(raw) < 0.0
    col = np.where(clamp, 0.0, raw)

    ar, br, cr = np.real(a), np.real(b), np.real(c)
    lam = 0.5 * (ar + cr) + np.sqrt(0.25 * (ar - cr) ** 2 + br * br)
    radius = np.ceil(3.0 * np.sqrt(lam)).astype(np.int64)
    visible = (np.real(tz) > NEAR) & (np.real(det) > 0.0)

    y = np.stack([mx, my, A, B, C, opac, col[0], col[1], col[2]])
    return dict(y=y, z=tz, radius=radius, visible=visible, clamp=clamp, Y=Y, dirs=dirs)


def tile_grid(W: int, H: int, TW: int, TH: int) -> tuple[int, int]:
    return -(-W // TW), -(-H // TH)


def rasterize_view(y: np.ndarray, lists: list, W: int, H: int, TW: int, TH: int) -> dict:
    """Front-to-back alpha-blending (eq. alpha-blending) of every pixel of one
    view, walking its tile's depth-sorted list; vectorised over all pixels.

    Per pixel centre p and splat with mean m, conic (A,B,C), opacity o:
    d = p - m, power = -0.5*(A dx^2 + C dy^2) - B dx dy; skip if power > 0;
    alpha = min(0.99, o*exp(power)); skip if alpha < 1/255; stop (without
    this splat) if T*(1 - alpha) < 1e-4; otherwise C += c*alpha*T and
    T *= 1 - alpha.  Background is black.

    Returns the image [3,H,W] and the contributing (pixel, splat) pairs in
    blending order with alpha, T, G = exp(power), the clamp flag and d.
    """
    y = np.real(y).astype(np.float64)
    TX, TY = tile_grid(W, H, TW, TH)
    nt = TX * TY
    npx = TW * TH
    maxlen = max((len(l) for l in lists), default=0)
    pad = np.full((nt, max(maxlen, 1)), -1, dtype=np.int64)
    for t, l in enumerate(lists):
        pad[t, :len(l)] = l
    tx = np.arange(nt) % TX
    ty = np.arange(nt) // TX
    lx = np.arange(npx) % TW
    ly = np.arange(npx) // TW
    pxi = tx[:, None] * TW + lx[None, :]                    # [nt, npx] integer pixel x
    pyi = ty[:, None] * TH + ly[None, :]
    pvalid = (pxi < W) & (pyi < H)
    px = pxi + 0.5
    py = pyi + 0.5
    T = np.ones((nt, npx))
    Cacc = np.zeros((3, nt, npx))
    done = ~pvalid
    ncontrib = np.zeros((nt, npx), dtype=np.int64)
    rec = {k: [] for k in ("tile", "lpix", "g", "order", "alpha", "T", "G", "clamped", "dx", "dy")}
    for k in range(maxlen):
        if done.all():
            break
        g = pad[:, k]
        has = g >= 0
        gs = np.where(has, g, 0)
        mx, my, A, B, C, o = (y[i][gs][:, None] for i in range(6))
        col = y[6:9][:, gs][:, :, None]                     # [3, nt, 1]
        dx = px - mx
        dy = py - my
        power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
        G = np.exp(np.minimum(power, 0.0))
        a_raw = o * G
        alpha = np.minimum(ALPHA_MAX, a_raw)
        cand = has[:, None] & ~done & (power <= 0.0) & (alpha >= ALPHA_MIN)
        Tn = T * (1.0 - alpha)
        stop = cand & (Tn < T_MIN)
        done = done | stop
        use = cand & ~stop
        if use.any():
            ti, pi = np.nonzero(use)
            rec["tile"].append(ti)
            rec["lpix"].append(pi)
            rec["g"].append(g[ti])
            rec["order"].append(np.full(len(ti), k))
            rec["alpha"].append(alpha[ti, pi])
            rec["T"].append(T[ti, pi])
            rec["G"].append(G[ti, pi])
            rec["clamped"].append(a_raw[ti, pi] > ALPHA_MAX)
            rec["dx"].append(dx[ti, pi])
            rec["dy"].append(dy[ti, pi])
            Cacc = Cacc + np.where(use[None], col * alpha[None] * T[None], 0.0)
            T = np.where(use, Tn, T)
            ncontrib += use
    pairs = {k: (np.concatenate(v) if v else np.zeros(0)) for k, v in rec.items()}
    for k in ("tile", "lpix", "g", "order"):
        pairs[k] = pairs[k].astype(np.int64)
    pairs["clamped"] = pairs["clamped"].astype(bool)
    gx = tx[pairs["tile"]] * TW + pairs["lpix"] % TW
    gy = ty[pairs["tile"]] * TH + pairs["lpix"] // TW
    pairs["pixel"] = gy * W + gx
    img = np.zeros((3, H * W))
    Tfin = np.ones(H * W)
    nc = np.zeros(H * W, dtype=np.int64)
    flat = (pyi * W + pxi)[pvalid]
    img[:, flat] = Cacc[:, pvalid]
    Tfin[flat] = T[pvalid]
    nc[flat] = ncontrib[pvalid]
    # d C / d alpha_k = T_k c_k - S_k / (1 - alpha_k), S_k = sum of c_j alpha_j T_j
    # over the later contributors j of the same pixel (plus T_final * background = 0).
    npair = len(pairs["g"])
    D = np.zeros((npair, 3))
    if npair:
        w = y[6:9][:, pairs["g"]].T * (pairs["alpha"] * pairs["T"])[:, None]    # [npair,3]
        # visit each pixel's contributors back to front and accumulate
        srt = np.lexsort((-pairs["order"], pairs["pixel"]))
        ws = w[srt]
        pix_s = pairs["pixel"][srt]
        first = np.concatenate([[True], pix_s[1:] != pix_s[:-1]])
        csum = np.cumsum(ws, axis=0)
        first_idx = np.nonzero(first)[0]
        before = np.vstack([np.zeros((1, 3)), csum[first_idx[1:] - 1]])
        incl = csum - before[np.cumsum(first) - 1]      # this and all later contributors
        S = np.empty_like(ws)
        S[srt] = incl - ws                              # later contributors only
        D = y[6:9][:, pairs["g"]].T * pairs["T"][:, None] - S / (1.0 - pairs["alpha"])[:, None]
    pairs["D"] = D
    return dict(image=img.reshape(3, H, W), T_final=Tfin.reshape(H, W),
                n_contrib=nc.reshape(H, W), pairs=pairs, TX=TX, TY=TY)


def render(x: np.ndarray, cams, deg: int, TW: int = 16, TH: int = 16) -> list[dict]:
    """Project, bin and blend every view of a camera set (Cameras-like object
    with .V and .view(v)).  Returns one dict per view."""
    out = []
    x64 = np.asarray(x, dtype=np.float64)
    for v in range(cams.V):
        cam = cams.view(v)
        pr = project(x64, cam, deg)
        bn = bin_view(pr["y"], pr["z"], pr["radius"], pr["visible"], cam["W"], cam["H"], TW, TH)
        rs = rasterize_view(pr["y"], bn["lists"], cam["W"], cam["H"], TW, TH)
        out.append(dict(proj=pr, bins=bn, raster=rs, cam=cam))
    return out


def render_images(x: np.ndarray, cams, deg: int, TW: int = 16, TH: int = 16) -> list[np.ndarray]:
    return [r["raster"]["image"] for r in render(x, cams, deg, TW, TH)]


def bin_view(y, z, radius, visible, W, H, TW, TH):
    """Tile binning and depth sort for one view (section 3.1: the
    rasteriser of 3DGS duplicates each splat into every tile its 3-sigma
    square touches and sorts the copies by tile and depth).

    Integer function of float32 records: the mean and depth are rounded to
    float32, the tile rectangle is floor((m -/+ r) / tile) evaluated in
    float32 (IEEE division) with inclusive bounds, and each tile's list is
    every splat whose rectangle holds the tile, ordered by (float32 depth
    bits, Gaussian id).  Returns the per-tile lists, their concatenation in
    tile order and the tile ranges."""
    TX, TY = tile_grid(W, H, TW, TH)
    f32 = np.float32
    mx = np.real(y[0]).astype(f32)
    my = np.real(y[1]).astype(f32)
    zb = np.real(z).astype(f32).view(np.uint32).astype(np.uint64)
    rr = radius.astype(f32)
    with np.errstate(invalid="ignore", over="ignore"):
        fx0 = np.floor((mx - rr) / f32(TW))
        fx1 = np.floor((mx + rr) / f32(TW))
        fy0 = np.floor((my - rr) / f32(TH))
        fy1 = np.floor((my + rr) / f32(TH))
    x0 = np.minimum(np.maximum(fx0, f32(0)), f32(TX)).astype(np.int64)
    x1 = np.maximum(np.minimum(fx1, f32(TX - 1)), f32(-1)).astype(np.int64)
    y0 = np.minimum(np.maximum(fy0, f32(0)), f32(TY)).astype(np.int64)
    y1 = np.maximum(np.minimum(fy1, f32(TY - 1)), f32(-1)).astype(np.int64)
    ok = visible & (x0 <= x1) & (y0 <= y1)
    gs = np.nonzero(ok)[0]
    w = (x1 - x0 + 1)[gs]
    h = (y1 - y0 + 1)[gs]
    cnt = w * h
    rep = np.repeat(gs, cnt)
    local = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ww = np.repeat(w, cnt)
    kt = (y0[rep] + local // ww) * TX + (x0[rep] + local % ww)
    ntiles = TX * TY
    kz = zb[rep]
    order = np.lexsort((rep, kz, kt))
    kt, kg = kt[order], rep[order]
    counts = np.bincount(kt, minlength=ntiles)
    starts = np.concatenate([[0], np.cumsum(counts)])
    lists = [kg[starts[i]:starts[i + 1]] for i in range(ntiles)]
    return dict(lists=lists, values=kg, tile_of_key=kt, ranges=starts, TX=TX, TY=TY,
                rect=np.stack([x0, y0, x1, y1]), binned=ok)
