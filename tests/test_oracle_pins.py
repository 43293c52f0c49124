"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, library routines, finite differences, brute force), chosen so
that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.  CPU only."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import forward, jacobian, solve
from oracle.sh import sh_basis
from paper_2409_12892_amd import scenegen as sg


# ---------------------------------------------------------------- helpers
def axis_camera(W=64, H=64, f=50.0, dist=4.0):
    """Camera at (0,0,-dist) looking along +z (identity rotation)."""
    return dict(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, dist], np.float32),
                fx=np.float32(f), fy=np.float32(f), cx=np.float32(W / 2), cy=np.float32(H / 2), W=W, H=H)


class OneCam:
    def __init__(self, cam):
        self.cam = cam
        self.V = 1

    def view(self, v):
        return self.cam


def small_scene(N, deg, seed, logscale_mu=-1.6, half=0.45):
    sc, rng = sg.make_scene(N, deg, seed, mean_lo=-half, mean_hi=half, logscale_mu=logscale_mu,
                            logscale_sigma=0.2)
    return sc, rng


# ---------------------------------------------------------------- SH basis
def real_sh_scipy(l, m, d):
    """Standard real SH from scipy's complex harmonics (which include the
    Condon-Shortley phase): Y_lm = sqrt2 (-1)^m Re/Im Y_l^|m|."""
    x, y, z = d
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    Yc = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Yc.real
    if m < 0:
        return math.sqrt(2) * (-1) ** m * Yc.imag
    return Yc.real


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(3, 200))
    d /= np.linalg.norm(d, axis=0)
    Y = sh_basis(d, 3)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[k], real_sh_scipy(l, m, d), rtol=0, atol=1e-13,
                                       err_msg=f"l={l} m={m}")
            k += 1


# ---------------------------------------------------------------- projection closed forms
def _one_gaussian(mean, logscale, quat, opac_logit, sh):
    K = sh.shape[0]
    x = np.zeros((11 + 3 * K, 1))
    x[0:3, 0] = mean
    x[3:6, 0] = logscale
    x[6:10, 0] = quat
    x[10, 0] = opac_logit
    x[11:, 0] = sh.reshape(-1)
    return x


def test_projection_isotropic_on_axis():
    cam = axis_camera(W=64, H=48, f=50.0, dist=4.0)
    s = math.log(0.05)
    sh = np.array([[0.3, -0.2, 0.1]])
    x = _one_gaussian([0, 0, 0], [s, s, s], [1, 0, 0, 0], 0.7, sh)
    pr = forward.project(x, cam, 0)
    y = pr["y"][:, 0]
    var = (50.0 * 0.05 / 4.0) ** 2 + 0.3
    assert y[0] == pytest.approx(32.0, abs=1e-12) and y[1] == pytest.approx(24.0, abs=1e-12)
    np.testing.assert_allclose(y[2:5], [1 / var, 0.0, 1 / var], rtol=1e-13, atol=1e-15)
    assert y[5] == pytest.approx(1 / (1 + math.exp(-0.7)), rel=1e-14)
    np.testing.assert_allclose(y[6:9], 0.5 + 0.28209479177387814 * sh[0], rtol=1e-14)
    assert pr["radius"][0] == math.ceil(3 * math.sqrt(var))
    assert pr["z"][0] == pytest.approx(4.0)


def test_projection_rotated_anisotropic_on_axis():
    """Rotation by theta about the optical axis: the screen covariance is the
    2D rotation of diag(s1^2, s2^2) scaled by (f/z)^2, plus the dilation."""
    cam = axis_camera(W=64, H=64, f=40.0, dist=5.0)
    th = 0.6
    s1, s2, s3 = 0.08, 0.03, 0.05
    x = _one_gaussian([0, 0, 0], np.log([s1, s2, s3]), [math.cos(th / 2), 0, 0, math.sin(th / 2)],
                      0.0, np.zeros((1, 3)))
    y = forward.project(x, cam, 0)["y"][:, 0]
    R2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    cov = (40.0 / 5.0) ** 2 * R2 @ np.diag([s1 ** 2, s2 ** 2]) @ R2.T + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov)
    np.testing.assert_allclose(y[2:5], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)


def test_projection_off_axis_mean_and_jacobian():
    """Off-axis mean: m = f t/z + c, and the screen covariance uses the
    perspective Jacobian at t (checked against a finite-difference Jacobian
    of the pinhole map applied to the 3D covariance)."""
    cam = axis_camera(W=100, H=80, f=70.0, dist=4.0)
    mean = np.array([0.4, -0.3, 0.2])
    ls = np.log([0.05, 0.1, 0.02])
    q = np.array([0.9, 0.2, -0.3, 0.25])
    x = _one_gaussian(mean, ls, q, 0.0, np.zeros((1, 3)))
    y = forward.project(x, cam, 0)["y"][:, 0]
    t = mean + np.array([0, 0, 4.0])
    assert y[0] == pytest.approx(70 * t[0] / t[2] + 50, rel=1e-14)
    assert y[1] == pytest.approx(70 * t[1] / t[2] + 40, rel=1e-14)

    def pin(p):
        return np.array([70 * p[0] / p[2], 70 * p[1] / p[2]])
    Jfd = np.stack([(pin(t + h) - pin(t - h)) / 2e-6 for h in np.eye(3) * 1e-6], axis=1)
    qn = q / np.linalg.norm(q)
    w, a, b, c = qn
    R = np.array([[1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b)],
                  [2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a)],
                  [2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)]])
    # R must be a proper rotation
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert np.linalg.det(R) == pytest.approx(1.0)
    S = R @ np.diag(np.exp(2 * ls)) @ R.T
    cov = Jfd @ S @ Jfd.T + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov)
    np.testing.assert_allclose(y[2:5], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-7)


def test_quaternion_rotation_direction():
    """q = (cos th/2, 0, 0, sin th/2) rotates counter-clockwise about +z."""
    th = 0.3
    R = forward.quat_to_rot(np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)]))
    np.testing.assert_allclose(R, [[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0],
                                   [0, 0, 1]], atol=1e-15)


# ---------------------------------------------------------------- blending closed forms
def _splats(rows):
    """y array from rows of (mx, my, A, B, C, o, r, g, b)."""
    return np.asarray(rows, np.float64).T


def test_blend_one_splat_closed_form():
    y = _splats([[8.5, 8.5, 0.02, 0.0, 0.02, 0.6, 0.2, 0.5, 0.9]])
    rs = forward.rasterize_view(y, [np.array([0])], 16, 16, 16, 16)
    p = rs["pairs"]
    # pixel (8, 8) sits exactly on the mean: alpha = o, C = c * o, dC/dalpha = c
    k = np.nonzero(p["pixel"] == 8 * 16 + 8)[0][0]
    assert p["alpha"][k] == pytest.approx(0.6)
    np.testing.assert_allclose(rs["image"][:, 8, 8], [0.2 * 0.6, 0.5 * 0.6, 0.9 * 0.6], rtol=1e-15)
    np.testing.assert_allclose(p["D"][k], [0.2, 0.5, 0.9], rtol=1e-13)
    assert p["T"][k] == 1.0


def test_blend_two_splats_closed_form():
    c1 = np.array([0.9, 0.1, 0.3])
    c2 = np.array([0.2, 0.7, 0.4])
    y = _splats([[4.5, 4.5, 0.05, 0.01, 0.04, 0.5, *c1],
                 [5.5, 3.5, 0.03, -0.01, 0.06, 0.8, *c2]])
    rs = forward.rasterize_view(y, [np.array([0, 1])], 8, 8, 8, 8)
    p = rs["pairs"]
    pix = 2 * 8 + 3          # pixel (3, 2)
    k1 = np.nonzero((p["pixel"] == pix) & (p["g"] == 0))[0][0]
    k2 = np.nonzero((p["pixel"] == pix) & (p["g"] == 1))[0][0]
    a1, a2 = p["alpha"][k1], p["alpha"][k2]
    # alpha from the definition
    d1 = np.array([3.5 - 4.5, 2.5 - 4.5])
    assert a1 == pytest.approx(0.5 * math.exp(-0.5 * (0.05 * d1[0] ** 2 + 0.04 * d1[1] ** 2)
                                              - 0.01 * d1[0] * d1[1]), rel=1e-14)
    np.testing.assert_allclose(rs["image"][:, 2, 3], c1 * a1 + c2 * a2 * (1 - a1), rtol=1e-14)
    np.testing.assert_allclose(p["D"][k1], c1 - c2 * a2, rtol=1e-13)
    np.testing.assert_allclose(p["D"][k2], (1 - a1) * c2, rtol=1e-13)
    assert p["T"][k2] == pytest.approx(1 - a1, rel=1e-15)


def test_blend_thresholds():
    """alpha clamp at 0.99, skip below 1/255, stop when T would fall below 1e-4."""
    # opacity 0.999 on the pixel centre: alpha clamped to 0.99, derivative flag set
    y = _splats([[0.5, 0.5, 1.0, 0.0, 1.0, 0.999, 1, 1, 1]] * 3)
    rs = forward.rasterize_view(y, [np.array([0, 1, 2])], 4, 4, 4, 4)
    p = rs["pairs"]
    at0 = p["pixel"] == 0
    # 1st: T 1 -> 0.01, 2nd: T would be 1e-4 (not < 1e-4) -> kept, 3rd: 1e-6 -> stop
    assert at0.sum() == 2
    assert p["alpha"][at0][0] == pytest.approx(0.99) and p["clamped"][at0].all()
    assert rs["T_final"][0, 0] == pytest.approx(1e-4)
    # a splat whose alpha at a pixel is below 1/255 does not contribute there
    y2 = _splats([[0.5, 0.5, 1.0, 0.0, 1.0, 0.5, 1, 1, 1]])
    rs2 = forward.rasterize_view(y2, [np.array([0])], 8, 8, 8, 8)
    q = rs2["pairs"]
    o_at = 0.5 * np.exp(-0.5 * ((q["dx"]) ** 2 + (q["dy"]) ** 2))
    assert (o_at >= 1 / 255).all()
    # brute-force count of pixels with alpha >= 1/255
    xs, ys = np.meshgrid(np.arange(8) + 0.5, np.arange(8) + 0.5)
    a_all = 0.5 * np.exp(-0.5 * ((xs - 0.5) ** 2 + (ys - 0.5) ** 2))
    assert len(q["g"]) == int((a_all >= 1 / 255).sum())


def test_suffix_sums_brute_force():
    """dC/dalpha from the vectorised suffix sums equals a per-pixel loop."""
    sc, rng = small_scene(24, 0, 11)
    cams = sg.fibonacci_cameras(1, 32, 32)
    vw = forward.render(sc.x, cams, 0)[0]
    p = vw["raster"]["pairs"]
    y = vw["proj"]["y"]
    for pix in np.unique(p["pixel"])[:50]:
        idx = np.nonzero(p["pixel"] == pix)[0]
        idx = idx[np.argsort(p["order"][idx])]
        for n, k in enumerate(idx):
            later = sum(y[6:9, p["g"][j]] * p["alpha"][j] * p["T"][j] for j in idx[n + 1:])
            expect = y[6:9, p["g"][k]] * p["T"][k] - later / (1 - p["alpha"][k])
            np.testing.assert_allclose(p["D"][k], expect, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- binning brute force
def _rect_members(pr, t, TX, TW, TH):
    mx = pr["y"][0].astype(np.float32).astype(np.float64)
    my = pr["y"][1].astype(np.float32).astype(np.float64)
    r = pr["radius"].astype(np.float64)
    zb = pr["z"].astype(np.float32).view(np.uint32)
    tx, ty = t % TX, t // TX
    # interval overlap of [m - r, m + r] with the half-open tile [x0, x0 + TW)
    inside = (pr["visible"] & (mx + r >= tx * TW) & (mx - r < (tx + 1) * TW)
              & (my + r >= ty * TH) & (my - r < (ty + 1) * TH))
    members = np.nonzero(inside)[0]
    return members[np.lexsort((members, zb[members]))]


def _quotient_margin(mx, my, r, TW, TH):
    """Distance of the four rectangle quotients (m -/+ r) / tile from the
    nearest integer: below 1e-5 the float32 floor may differ from the exact
    interval test."""
    qs = np.array([(mx - r) / TW, (mx + r) / TW, (my - r) / TH, (my + r) / TH])
    return float(np.min(np.abs(qs - np.round(qs))))


def test_binning_brute_force():
    """Every tile list is the set of splats whose 3-sigma rectangle covers
    the tile (an interval test per splat and tile), in (depth, id) order;
    the key count equals the summed rectangle areas."""
    d = sg.config_scene("tiny", N=300)
    cams = d["cams"][0]
    for v in range(cams.V):
        cam = cams.view(v)
        for TW, TH in ((16, 16), (8, 16), (16, 8), (32, 8), (8, 32)):
            pr = forward.project(d["scene"].x.astype(np.float64), cam, 0)
            bn = forward.bin_view(pr["y"], pr["z"], pr["radius"], pr["visible"], 64, 64, TW, TH)
            mx = pr["y"][0].astype(np.float32).astype(np.float64)
            my = pr["y"][1].astype(np.float32).astype(np.float64)
            r = pr["radius"].astype(np.float64)
            zb = pr["z"].astype(np.float32).view(np.uint32)
            TX, TY = bn["TX"], bn["TY"]
            total = 0
            for t in range(TX * TY):
                members = _rect_members(pr, t, TX, TW, TH)
                got = bn["lists"][t]
                # a difference is only acceptable at a float32 rounding margin of the quotient
                for g in np.setxor1d(got, members):
                    assert _quotient_margin(mx[g], my[g], r[g], TW, TH) < 1e-5, (t, g)
                same = np.intersect1d(got, members)
                np.testing.assert_array_equal(got[np.isin(got, same)], members[np.isin(members, same)])
                total += len(got)
                zs = zb[got]
                assert np.all((zs[1:] > zs[:-1]) | ((zs[1:] == zs[:-1]) & (got[1:] > got[:-1])))
            rect = bn["rect"][:, bn["binned"]]
            assert total == len(bn["values"])
            assert total == int(((rect[2] - rect[0] + 1) * (rect[3] - rect[1] + 1)).sum())


def _below_threshold_everywhere(pr, g, t, TX, TW, TH, W, H):
    """True when splat g has alpha = o exp(power) < 1/255 at every pixel
    centre of tile t inside the image (eq. alpha-blending then skips it at
    every pixel of the tile)."""
    y = np.real(pr["y"])
    tx, ty = t % TX, t // TX
    px = tx * TW + np.arange(TW)
    py = ty * TH + np.arange(TH)
    px, py = px[px < W] + 0.5, py[py < H] + 0.5
    dx = px[None, :] - y[0, g]
    dy = py[:, None] - y[1, g]
    power = -0.5 * (y[2, g] * dx * dx + y[4, g] * dy * dy) - y[3, g] * dx * dy
    return bool((y[5, g] * np.exp(power) < forward.ALPHA_MIN).all())


def test_keys_below_the_alpha_threshold_do_not_change_the_blend():
    """Leaving out of a tile's list the splats that stay below the alpha
    threshold at every pixel centre of the tile (checked pixel by pixel)
    gives the same image and the same contributing pairs, bit for bit: the
    blend of eq. alpha-blending skips them, so a rasteriser may omit such
    (splat, tile) keys."""
    d = sg.config_scene("tiny", N=400)
    cams = d["cams"][0]
    n_out = 0
    for v in range(2):
        cam = cams.view(v)
        W, H = cam["W"], cam["H"]
        for TW, TH in ((16, 16), (8, 32)):
            pr = forward.project(d["scene"].x.astype(np.float64), cam, 0)
            bn = forward.bin_view(pr["y"], pr["z"], pr["radius"], pr["visible"], W, H, TW, TH)
            TX = bn["TX"]
            thin = []
            for t, lst in enumerate(bn["lists"]):
                keep = np.array([not _below_threshold_everywhere(pr, g, t, TX, TW, TH, W, H) for g in lst], bool)
                n_out += int((~keep).sum())
                thin.append(lst[keep])
            a = forward.rasterize_view(pr["y"], thin, W, H, TW, TH)
            b = forward.rasterize_view(pr["y"], bn["lists"], W, H, TW, TH)
            np.testing.assert_array_equal(a["image"], b["image"])
            # the same (pixel, splat) pairs with the same state (enumeration order
            # follows list positions, so compare in (pixel, splat) order)
            sa = np.lexsort((a["pairs"]["g"], a["pairs"]["pixel"]))
            sb = np.lexsort((b["pairs"]["g"], b["pairs"]["pixel"]))
            for k in ("pixel", "g", "T", "alpha", "D"):
                np.testing.assert_array_equal(a["pairs"][k][sa], b["pairs"][k][sb])
    assert n_out > 0


# ---------------------------------------------------------------- whole-J finite differences
def _signature(views):
    out = []
    for vw in views:
        p = vw["raster"]["pairs"]
        out.append((p["pixel"].tobytes(), p["g"].tobytes(), p["order"].tobytes(), p["clamped"].tobytes()))
    return out


@pytest.mark.parametrize("deg,N,seed", [(0, 24, 5), (3, 8, 6)])
def test_jacobian_finite_differences(deg, N, seed):
    sc, rng = small_scene(N, deg, seed)
    cams = sg.fibonacci_cameras(1, 32, 32)
    x = sc.x.astype(np.float64)
    J = jacobian.Jacobian(x, cams, deg)
    sig0 = _signature(J.views)
    Jd = J.J.toarray()
    checked = 0
    for j in range(x.shape[0]):
        for g in range(x.shape[1]):
            h = 1e-6 * max(1.0, abs(x[j, g]))
            xp = x.copy(); xp[j, g] += h
            xm = x.copy(); xm[j, g] -= h
            vp = forward.render(xp, cams, deg)
            vm = forward.render(xm, cams, deg)
            if _signature(vp) != sig0 or _signature(vm) != sig0:
                continue          # active set changes across the step: not differentiable here
            fd = (vp[0]["raster"]["image"].ravel() - vm[0]["raster"]["image"].ravel()) / (2 * h)
            col = Jd[:, j * x.shape[1] + g]
            # central-difference truncation is O(h^2) ~ 1e-12; rounding noise of the
            # difference quotient is ~ eps / h ~ 1e-10 per pixel, hence the floor
            err = np.linalg.norm(col - fd)
            assert err < 1e-6 * np.linalg.norm(fd) + 1e-9, (j, g, err, np.linalg.norm(fd))
            checked += 1
    assert checked > 0.8 * x.size


# ---------------------------------------------------------------- J^T J structure
def _tiny_problem(deg=0, N=40, seed=7, V=2, size=32):
    sc, rng = small_scene(N, deg, seed)
    cams = sg.fibonacci_cameras(V, size, size)
    J = jacobian.Jacobian(sc.x, cams, deg)
    return sc, cams, J


def test_jtj_symmetric_psd_adjoint_and_diag():
    sc, cams, J = _tiny_problem()
    A = J.JtJ().toarray()
    assert np.abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= -1e-12 * ev.max()
    rng = np.random.default_rng(3)
    p = rng.normal(size=J.P * J.N)
    u = rng.normal(size=J.n_res)
    Jp = J.apply_J(p)
    assert abs(Jp @ u - p @ J.apply_JT(u)) <= 1e-12 * np.linalg.norm(Jp) * np.linalg.norm(u)
    assert p @ J.apply_JtJ(p) == pytest.approx(Jp @ Jp, rel=1e-12)
    diag = J.diag_JtJ()
    Jd = J.J.toarray()
    for j in range(0, J.P * J.N, 7):
        assert diag[j] == pytest.approx(float(Jd[:, j] @ Jd[:, j]), rel=1e-13, abs=1e-300)
    np.testing.assert_allclose(np.diag(A), diag, rtol=1e-13)


def test_pcg_matches_dense_solve():
    sc, cams, J = _tiny_problem(seed=8)
    rng = np.random.default_rng(4)
    targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
    b = J.b(targets)
    M = J.diag_JtJ()
    lam = 1e-2
    ref = solve.dense_solve(J.JtJ(), b, lam)
    out = solve.pcg(J.apply_JtJ, b, M, lam, n_iters=2000, tol=1e-13, tol_mode=solve.TOL_RELATIVE)
    assert np.linalg.norm(out["x"] - ref) / np.linalg.norm(ref) < 1e-8


def test_pcg_with_diag_floor_matches_dense_solve():
    """The minimum-diagonal variant solves (J^T J + lam max(diag, floor)) d = b."""
    sc, cams, J = _tiny_problem(seed=8)
    rng = np.random.default_rng(4)
    targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
    b = J.b(targets)
    M = J.diag_JtJ()
    floor = float(np.quantile(M[M > 0], 0.3))
    ref = solve.dense_solve(J.JtJ(), b, 0.1, diag_floor=floor)
    out = solve.pcg(J.apply_JtJ, b, M, 0.1, n_iters=2000, tol=1e-13, tol_mode=solve.TOL_RELATIVE,
                    diag_floor=floor)
    assert np.linalg.norm(out["x"] - ref) / np.linalg.norm(ref) < 1e-8
    plain = solve.dense_solve(J.JtJ(), b, 0.1)
    assert np.linalg.norm(plain - ref) / np.linalg.norm(ref) > 1e-3     # the floor matters here
    # x0 of Algorithm 1 uses the floored diagonal
    one = solve.pcg(J.apply_JtJ, b, M, 0.1, n_iters=0, diag_floor=floor)
    Mf = np.where(M > 0, np.maximum(M, floor), 0.0)
    np.testing.assert_allclose(one["x"], solve.jacobi_inverse(Mf) * b, rtol=1e-15)


def test_pcg_applies_count_and_history():
    sc, cams, J = _tiny_problem(seed=9)
    b = J.b([np.zeros_like(im) for im in J.images()])
    M = J.diag_JtJ()
    calls = []

    def A(p):
        calls.append(1)
        return J.apply_JtJ(p)
    out = solve.pcg(A, b, M, 1e-2, n_iters=8)
    assert len(calls) == 9 and out["iters"] == 8 and len(out["history"]) == 9


def _disjoint_colour_problem(V=2, deg=0):
    """Well separated Gaussians, so the colour columns never share a pixel."""
    N = 9
    x = np.zeros((sg.n_params(deg), N), np.float32)
    gx, gy = np.meshgrid([-0.6, 0.0, 0.6], [-0.6, 0.0, 0.6])
    x[0] = gx.ravel()
    x[1] = gy.ravel()
    x[3:6] = math.log(0.04)
    x[6] = 1.0
    x[10] = 0.5
    rng = np.random.default_rng(12)
    x[11:14] = rng.normal(0, 0.3, size=(3, N))
    # frontal cameras (identity rotation, small sideways shifts): the grid
    # never overlaps itself in projection
    V_ = V
    f32 = np.float32
    shifts = np.array([[0.05 * (v % 2), -0.04 * (v // 2), 4.0] for v in range(V_)], f32)
    cams = sg.Cameras(np.repeat(np.eye(3, dtype=f32)[None], V_, 0), shifts,
                      np.full(V_, 40, f32), np.full(V_, 40, f32), np.full(V_, 24, f32),
                      np.full(V_, 24, f32), np.full(V_, 48, np.int32), np.full(V_, 48, np.int32))
    return x, cams


def test_pcg_diagonal_system_exact_after_one_iteration():
    deg = 0
    x, cams = _disjoint_colour_problem()
    J = jacobian.Jacobian(x, cams, deg)
    N = x.shape[1]
    colour = np.zeros(J.P * N, bool)
    colour[11 * N:14 * N] = True
    Jc = J.J[:, np.nonzero(colour)[0]]
    A = (Jc.T @ Jc).toarray()
    assert np.abs(A - np.diag(np.diag(A))).max() == 0.0
    rng = np.random.default_rng(2)
    targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
    F = J.residual(targets)
    b = -(Jc.T @ F)
    M = np.diag(A).copy()
    lam = 0.3
    out = solve.pcg(lambda p: Jc.T @ (Jc @ p), b, M, lam, n_iters=1)
    expect = solve.jacobi_inverse(M) * b / (1 + lam)
    np.testing.assert_allclose(out["x"], expect, rtol=1e-12, atol=1e-300)


def test_linear_colour_special_case_recovers_perturbation():
    """Geometry frozen, SH degree 0: colour is linear in the DC coefficients,
    so one exact Gauss-Newton step (lambda -> 0) recovers a DC perturbation."""
    deg = 0
    sc, rng = small_scene(30, deg, 21)
    cams = sg.fibonacci_cameras(3, 40, 40)
    x = sc.x.astype(np.float64)
    dc = np.zeros_like(x)
    dc[11:14] = rng.normal(0, 0.03, size=(3, x.shape[1]))
    targets = forward.render_images(x + dc, cams, deg)
    J = jacobian.Jacobian(x, cams, deg)
    assert not any(vw["proj"]["clamp"].any() for vw in J.views)
    N = x.shape[1]
    cols = np.arange(11 * N, 14 * N)
    Jc = J.J[:, cols].toarray()
    b = -(Jc.T @ J.residual(targets))
    A = Jc.T @ Jc
    obs = np.diag(A) > 1e-12
    delta = np.linalg.solve(A[np.ix_(obs, obs)], b[obs])
    np.testing.assert_allclose(delta, dc[11:14].ravel()[obs], rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- subset combination
def test_combine_single_subset_identity():
    rng = np.random.default_rng(0)
    d = rng.normal(size=50)
    M = np.abs(rng.normal(size=50))
    M[::7] = 0
    out = solve.combine_subsets([d], [M])
    np.testing.assert_allclose(out[M > 0], d[M > 0], rtol=1e-15)
    assert np.all(out[M == 0] == 0)


def test_combine_equals_joint_solve_when_diagonal():
    """Supplement B: with diagonal J_i^T J_i the weighted mean is exact."""
    deg = 0
    x, cams = _disjoint_colour_problem(V=4)
    N = x.shape[1]
    cols = np.arange(11 * N, 14 * N)
    rng = np.random.default_rng(5)
    subsets = [cams.subset([0, 1]), cams.subset([2, 3])]
    deltas, Ms, As, bs = [], [], [], []
    for cs in subsets:
        J = jacobian.Jacobian(x, cs, deg)
        targets = [im + rng.normal(0, 0.05, size=im.shape) for im in J.images()]
        Jc = J.J[:, cols]
        A = (Jc.T @ Jc).toarray()
        b = -(Jc.T @ J.residual(targets))
        M = np.diag(A).copy()
        deltas.append(solve.jacobi_inverse(M) * b)     # exact solve of a diagonal system
        Ms.append(M)
        As.append(A)
        bs.append(b)
    joint = np.zeros_like(bs[0])
    Aj = As[0] + As[1]
    obs = np.diag(Aj) > 0
    joint[obs] = np.linalg.solve(Aj[np.ix_(obs, obs)], (bs[0] + bs[1])[obs])
    np.testing.assert_allclose(solve.combine_subsets(deltas, Ms), joint, rtol=1e-12, atol=1e-300)


# ---- low-precision cache: rounding of the stored T and dC/dalpha ----

def test_bf16_rounding_ties_to_even_and_error_bound():
    from oracle.jacobian import round_bf16
    one = 1.0
    cases = {one: one, one + 2.0 ** -8: one,                       # tie -> even (1.0)
             one + 3 * 2.0 ** -8: one + 2.0 ** -6,                 # tie between odd and even -> even
             one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,        # above the tie
             -2.5: -2.5, 0.0: 0.0}
    for v, ref in cases.items():
        assert round_bf16(np.array([v]))[0] == ref, v
    rng = np.random.default_rng(7)
    v = rng.uniform(-3, 3, 10000) * 10.0 ** rng.uniform(-4, 0, 10000)
    r = round_bf16(v)
    assert np.all(np.abs(r - v) <= 2.0 ** -8 * np.abs(v) * (1 + 1e-6))
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def test_f16_rounding_ties_to_even_and_error_bound():
    from oracle.jacobian import round_f16
    one = 1.0
    cases = {one + 2.0 ** -11: one, one + 3 * 2.0 ** -11: one + 2.0 ** -9, one + 2.0 ** -11 + 2.0 ** -20: one + 2.0 ** -10,
             1e-4: 1.0001659393310547e-04}       # 1e-4 = 0x068E in binary16 (normal)
    for v, ref in cases.items():
        assert round_f16(np.array([v]))[0] == ref, v
    rng = np.random.default_rng(8)
    v = rng.uniform(-3, 3, 10000) * 10.0 ** rng.uniform(-4, 0, 10000)
    v = v[np.abs(v) >= 2.0 ** -14]                    # normal range
    assert np.all(np.abs(round_f16(v) - v) <= 2.0 ** -11 * np.abs(v) * (1 + 1e-6))


def test_rounded_jacobian_within_storage_bound():
    """J(dtype) differs from J entry by entry by at most the storage rounding
    of T and D times their coefficients; the first splat of a pixel has
    T = 1, which every type stores exactly."""
    d = sg.config_scene("tiny", N=200, subsets=[(2, 32, 32)], seed=31)
    sc, cams = d["scene"], d["cams"][0]
    J = jacobian.Jacobian(sc.x, cams, sc.sh_degree)
    # relative half-ulp of the type, plus (binary16) half the subnormal spacing
    for dt, eps, tiny in (("f32", 2.0 ** -24, 0.0), ("bf16", 2.0 ** -8, 0.0), ("f16", 2.0 ** -11, 2.0 ** -25)):
        Jr = J.rounded(dt)
        assert Jr.J.nnz == J.J.nnz
        bound = (eps * 1.0001 + 2.0 ** -24) * (np.abs(J._D * J._geo) + np.abs(J._T * J._col)) + tiny * (
            np.abs(J._geo) + np.abs(J._col))
        exact = J._D * J._geo + J._T * J._col
        rnd = jacobian.CACHE_ROUNDING[dt]
        approx = rnd(J._D) * J._geo + rnd(J._T) * J._col
        assert np.all(np.abs(approx - exact) <= bound + 1e-300)
        # the rounded matrix holds exactly these values
        p = np.random.default_rng(3).normal(size=J.P * J.N)
        ref = np.zeros(J.n_res)
        np.add.at(ref, J._rows, approx * p[J._cols])
        np.testing.assert_allclose(Jr.apply_J(p), ref, rtol=1e-12, atol=1e-15)
    first = J._T == 1.0
    assert first.any()
    for dt in ("bf16", "f16"):
        assert np.all(jacobian.CACHE_ROUNDING[dt](J._T[first]) == 1.0)
