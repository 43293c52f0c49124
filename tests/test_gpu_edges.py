"""Edge cases of the HIP path against the oracle: a view that sees nothing,
a scene with no visible Gaussian (no keys, no pairs), a single Gaussian,
splats so large that one (Gaussian, view) owns more than 128 segments, and
option validation."""
import numpy as np
import pytest

from gpu_common import random_direction, rel
from oracle import forward, jacobian, solve
from paper_2409_12892_amd import scenegen as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def away_camera(cams: sg.Cameras, v: int) -> sg.Cameras:
    """Copy of camera v turned to look away from the scene (x and z axes
    flipped keep a proper rotation)."""
    R = cams.R[v].astype(np.float64)
    C = -R.T @ cams.t[v].astype(np.float64)
    R2 = np.diag([-1.0, 1.0, -1.0]) @ R
    t2 = -R2 @ C
    out = cams.subset([v])
    out.R = R2[None].astype(np.float32)
    out.t = t2[None].astype(np.float32)
    return out


def _run(scene, cams, target, tile=(16, 16)):
    from paper_2409_12892_amd import binding as B
    x = torch.from_numpy(scene.x).cuda()
    tgt = torch.from_numpy(np.ascontiguousarray(target).ravel()).cuda()
    cache, b, fsq = B.lm_build_cache(x, scene.sh_degree, cams, tgt, tile=tile)
    return B, x, cache, b, fsq


def test_view_facing_away_has_no_splats():
    d = sg.config_scene("tiny", N=600, subsets=[(3, 48, 48)], seed=21)
    sc = d["scene"]
    cams = sg.Cameras.concat([d["cams"][0].subset([0]), away_camera(d["cams"][0], 1), d["cams"][0].subset([2])])
    rng = np.random.default_rng(1)
    target = rng.uniform(0, 1, size=(3, 3, 48, 48)).astype(np.float32)
    J = jacobian.Jacobian(sc.x, cams, sc.sh_degree)
    assert len(J.views[1]["bins"]["values"]) == 0
    B, x, cache, b, fsq = _run(sc, cams, target)
    rngs = cache.export("tile_ranges")
    nt = 9
    assert rngs[nt] == rngs[2 * nt]                     # view 1: every tile list empty
    np.testing.assert_allclose(cache.export("residual").reshape(3, 3, 48, 48)[1], -target[1], atol=0)
    ref_b = J.b(list(target)).reshape(sc.P, -1)
    assert rel(b.cpu().numpy(), ref_b) < 1e-5
    p = random_direction(sc.P, sc.N, seed=3)
    # every residual is written, also those of pixels (and 8x8 blocks)
    # without pairs: the output starts as NaN
    out = torch.full((3 * 3 * 48 * 48,), float("nan"), device="cuda")
    u = B.lm_apply_J(cache, torch.from_numpy(p).cuda(), out=out).cpu().numpy()
    assert np.isfinite(u).all()
    assert rel(u, J.apply_J(p.astype(np.float64))) < 1e-5
    assert np.all(u.reshape(3, 3, 48, 48)[1] == 0)
    cache_t, _, _ = B.lm_build_cache(x, sc.sh_degree, cams, torch.from_numpy(target.ravel()).cuda(), thin_window=8)
    out.fill_(float("nan"))
    ut = B.lm_apply_J(cache_t, torch.from_numpy(p).cuda(), out=out).cpu().numpy()
    assert np.isfinite(ut).all() and np.all(ut.reshape(3, 3, 48, 48)[1] == 0)
    assert rel(ut, J.apply_J(p.astype(np.float64))) < 1e-5
    cache_t.destroy()


def test_no_visible_gaussian():
    d = sg.config_scene("tiny", N=64, subsets=[(2, 32, 32)], seed=22)
    sc = d["scene"]
    cams = sg.Cameras.concat([away_camera(d["cams"][0], 0), away_camera(d["cams"][0], 1)])
    target = np.full((2, 3, 32, 32), 0.25, np.float32)
    B, x, cache, b, fsq = _run(sc, cams, target)
    info = cache.info()
    assert info["n_keys"] == 0 and info["n_pairs"] == 0 and info["n_segments"] == 0
    assert float(fsq.item()) == pytest.approx(2 * 3 * 32 * 32 * 0.0625)
    assert torch.count_nonzero(b).item() == 0
    M = B.lm_jacobi_diag(cache)
    assert torch.count_nonzero(M).item() == 0
    deltas, stats = B.lm_pcg_solve([cache], [b], [M], 1e-2, 5)
    assert torch.count_nonzero(deltas[0]).item() == 0
    assert stats[0]["status"] == B.LM_WARN_BREAKDOWN and stats[0]["iters"] == 0
    ref = solve.pcg(lambda v: 0 * v, np.zeros(sc.P * sc.N), np.zeros(sc.P * sc.N), 1e-2, 5)
    assert ref["status"] == 1 and ref["iters"] == 0


def test_single_gaussian_sh3():
    sc, _ = sg.make_scene(1, 3, 23, mean_lo=-0.1, mean_hi=0.1, logscale_mu=-2.0)
    cams = sg.fibonacci_cameras(2, 32, 32)
    imgs = forward.render_images(sc.x, cams, 3)
    target = (np.stack(imgs) * 0.9).astype(np.float32)
    J = jacobian.Jacobian(sc.x, cams, 3)
    assert J.n_pairs > 0
    B, x, cache, b, fsq = _run(sc, cams, target)
    assert cache.info()["n_pairs"] == J.n_pairs
    assert rel(b.cpu().numpy().ravel(), J.b(list(target))) < 1e-5
    M = B.lm_jacobi_diag(cache).cpu().numpy().ravel()
    assert rel(M, J.diag_JtJ()) < 1e-5
    p = random_direction(sc.P, sc.N, seed=4)
    g = B.lm_apply_JtJ(cache, torch.from_numpy(p).cuda()).cpu().numpy().ravel()
    assert rel(g, J.apply_JtJ(p.astype(np.float64))) < 1e-5


def test_large_splats_span_many_tiles():
    """A few splats covering a whole 192x192 view (144 tiles): the segment
    list of one (Gaussian, view) crosses several 64-entry waves of the
    per-(Gaussian, view) reductions behind J^T u and diag(J^T J)."""
    sc, _ = sg.make_scene(6, 0, 25, mean_lo=-0.2, mean_hi=0.2, logscale_mu=0.0, logscale_sigma=0.1)
    cams = sg.fibonacci_cameras(1, 192, 192)
    imgs = forward.render_images(sc.x, cams, 0)
    target = (np.stack(imgs) * 0.8 + 0.05).astype(np.float32)
    J = jacobian.Jacobian(sc.x, cams, 0)
    B, x, cache, b, fsq = _run(sc, cams, target)
    info = cache.info()
    assert info["n_pairs"] == J.n_pairs
    assert info["n_segments"] > 3 * 64 and info["n_gv"] <= 6   # some gv owns > 128 segments
    assert rel(b.cpu().numpy().ravel(), J.b(list(target))) < 1e-5
    M = B.lm_jacobi_diag(cache).cpu().numpy().ravel()
    assert rel(M, J.diag_JtJ()) < 1e-5
    for seed in (5, 6):
        p = random_direction(sc.P, sc.N, seed=seed)
        g = B.lm_apply_JtJ(cache, torch.from_numpy(p).cuda()).cpu().numpy().ravel()
        assert rel(g, J.apply_JtJ(p.astype(np.float64))) < 1e-5


def test_invalid_options_are_rejected():
    from paper_2409_12892_amd import binding as B
    d = sg.config_scene("tiny", N=16, subsets=[(1, 16, 16)], seed=24)
    x = torch.from_numpy(d["scene"].x).cuda()
    tgt = torch.zeros(3 * 16 * 16, device="cuda")
    with pytest.raises(RuntimeError, match="tile_w"):
        B.lm_build_cache(x, 0, d["cams"][0], tgt, tile=(32, 16))
    with pytest.raises(RuntimeError, match="sh_degree"):
        B.lm_build_cache(x, 4, d["cams"][0], tgt)


def test_compact_build_keeps_the_products_and_refuses_build_exports():
    """LM_BUILD_COMPACT frees the build-only buffers: products, diagonal and
    per-view residuals are bit-identical to those of a full build, the pair
    arrays still export, the residual image does not (nor the objective,
    which reads it), and a rebuild on the compacted handle works."""
    from paper_2409_12892_amd import binding as B
    d = sg.config_scene("tiny", N=700, subsets=[(3, 64, 48)], seed=23, deg=1)
    sc, cams = d["scene"], d["cams"][0]
    imgs = forward.render_images(d["x_star"], cams, sc.sh_degree)
    tgt = torch.from_numpy(np.stack([(im + nz).astype(np.float32) for im, nz in zip(imgs, d["noise"][0])]).ravel()).cuda()
    x = torch.from_numpy(sc.x).cuda()
    full, b1, f1 = B.lm_build_cache(x, sc.sh_degree, cams, tgt)
    comp, b2, f2 = B.lm_build_cache(x, sc.sh_degree, cams, tgt, compact=True)
    assert torch.equal(b1, b2) and torch.equal(f1, f2)
    assert comp.info()["device_bytes"] < full.info()["device_bytes"]
    p = torch.from_numpy(random_direction(sc.P, sc.N, seed=5)).cuda()
    M1, M2 = B.lm_jacobi_diag(full), B.lm_jacobi_diag(comp)
    assert torch.equal(M1, M2)
    assert torch.equal(B.lm_apply_JtJ(full, p, 1e-2, M1), B.lm_apply_JtJ(comp, p, 1e-2, M2))
    assert torch.equal(B.lm_cache_view_sqnorm(full), B.lm_cache_view_sqnorm(comp))
    np.testing.assert_array_equal(full.export("pair_T"), comp.export("pair_T"))
    with pytest.raises(RuntimeError):
        comp.export("residual")
    with pytest.raises(RuntimeError):       # the objective needs the residual image
        B.lm_cache_objective(comp, tgt, B.objective())
    comp2, b3, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt, cache=comp)
    assert torch.equal(b3, b1)
    assert comp2.export("residual").size == 3 * 3 * 64 * 48
    full.destroy()
    comp2.destroy()


def test_compact_cache_drops_the_gram_transients_and_trims():
    """A compact cache keeps no per-(splat, tile) Gram values after the
    diagonal; lm_cache_trim frees the per-(Gaussian, view) Gram values too,
    PCG on the trimmed cache is bit-identical, and the diagonal and the
    learned-preconditioner inputs computed again are bit-identical."""
    from paper_2409_12892_amd import binding as B
    d = sg.config_scene("tiny", N=700, subsets=[(3, 64, 48)], seed=25, deg=1)
    sc, cams = d["scene"], d["cams"][0]
    x = torch.from_numpy(sc.x).cuda()
    tgt = B.lm_render(torch.from_numpy(d["x_star"]).cuda(), sc.sh_degree, cams)
    full, b1, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt)
    comp, b2, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt, compact=True)
    M1, M2 = B.lm_jacobi_diag(full), B.lm_jacobi_diag(comp)
    assert torch.equal(M1, M2)
    mf, mc = full.memory(), comp.memory()
    assert mf.get("gram", 0) > 0 and mc.get("gram", 0) == 0
    assert mc.get("gvgram", 0) > 0
    assert sum(mc.values()) == comp.info()["device_bytes"]
    f1 = B.lm_precond_features(comp, x, M2)
    d1, st1 = B.lm_pcg_solve([comp], [b2], [M2], 1e-2, 6)
    comp.trim()
    mt = comp.memory()
    assert mt.get("gvgram", 0) == 0 and mt.get("gram", 0) == 0
    assert comp.info()["device_bytes"] < sum(mc.values())
    d2, st2 = B.lm_pcg_solve([comp], [b2], [M2], 1e-2, 6)
    assert torch.equal(d1[0], d2[0])
    assert torch.equal(B.lm_jacobi_diag(comp), M1)
    assert torch.equal(B.lm_precond_features(comp, x, M2), f1)
    full.destroy()
    comp.destroy()


def test_compact_builds_share_a_scratch_handle():
    """Compact builds of two subsets through one scratch handle: products,
    diagonal and b are bit-identical to those of full builds; the compacted
    caches hold only what the products read, the scratch handle holds the
    transients and is no built cache."""
    from paper_2409_12892_amd import binding as B
    d = sg.config_scene("tiny", N=700, subsets=[(3, 64, 48), (2, 80, 40)], seed=24, deg=1)
    sc = d["scene"]
    x = torch.from_numpy(sc.x).cuda()
    scratch = B.Cache()
    for i, cams in enumerate(d["cams"]):
        print(f"[gpu edges] scratch-shared compact build, subset {i}", flush=True)
        imgs = forward.render_images(d["x_star"], cams, sc.sh_degree)
        tgt = torch.from_numpy(np.stack([(im + nz).astype(np.float32)
                                         for im, nz in zip(imgs, d["noise"][i])]).ravel()).cuda()
        full, b1, f1 = B.lm_build_cache(x, sc.sh_degree, cams, tgt)
        comp, b2, f2 = B.lm_build_cache(x, sc.sh_degree, cams, tgt, compact=True, scratch=scratch)
        assert torch.equal(b1, b2) and torch.equal(f1, f2)
        p = torch.from_numpy(random_direction(sc.P, sc.N, seed=6 + i)).cuda()
        M1, M2 = B.lm_jacobi_diag(full), B.lm_jacobi_diag(comp)
        assert torch.equal(M1, M2)
        assert torch.equal(B.lm_apply_JtJ(full, p, 1e-2, M1), B.lm_apply_JtJ(comp, p, 1e-2, M2))
        assert comp.info()["device_bytes"] < full.info()["device_bytes"]
        full.destroy()
        comp.destroy()
    assert scratch.handle.value
    with pytest.raises(RuntimeError):
        B.lm_jacobi_diag(scratch)
    scratch.destroy()
