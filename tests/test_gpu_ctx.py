"""Library contexts (include/lm3dgs.h lm_ctx_create): two contexts with
different allocators in one process - PyTorch's caching allocator and
hipMalloc - build the same cache and give the same results; per-context
graph mode and profiling; a context cannot be destroyed under its caches;
the fallback warnings; the vector steps of the LM loop.

Bit for bit: the cache arrays, the render, J p (each pixel's sum is added
in a fixed order).  The J^T products and the Jacobi diagonal add per-segment
sums from the waves of a tile into LDS with atomic adds whose order between
waves follows the scheduling, so they are compared within 1e-6."""
import numpy as np
import pytest

from gpu_common import make_problem, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _torch_allocator(B):
    used = []

    def _alloc(user, nbytes, stream):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
            used.append(int(nbytes))
            return p
        except Exception:
            return None

    def _free(user, ptr, stream):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    a = B.LmAllocator(None, B.LmAllocator._fields_[1][1](_alloc), B.LmAllocator._fields_[2][1](_free))
    return a, used


def test_two_contexts_with_different_allocators_agree():
    from paper_2409_12892_amd import binding as B
    pr = make_problem("tiny", deg=3, with_J=False)
    sc, cams = pr["scene"], pr["cams"]
    x = torch.from_numpy(sc.x).cuda()
    tgt = torch.from_numpy(pr["target"].ravel()).cuda()
    al, used = _torch_allocator(B)
    ctx_t = B.Ctx(al)
    ctx_h = B.Ctx(None)
    out = {}
    for name, ctx in (("torch", ctx_t), ("hip", ctx_h)):
        print(f"[ctx] build in the {name} context", flush=True)
        cache, b, fsq = B.lm_build_cache(x, sc.sh_degree, cams, tgt, ctx=ctx)
        M = B.lm_jacobi_diag(cache)
        p = torch.from_numpy(np.random.default_rng(3).normal(size=sc.x.shape).astype(np.float32)).cuda()
        u = B.lm_apply_J(cache, p)
        g = B.lm_apply_JtJ(cache, p, 0.1, M)
        d, st = B.lm_pcg_solve([cache], [b], [M], 1e-2, 8)
        out[name] = dict(vals=cache.export("sorted_values"), T=cache.export("pair_T"), D=cache.export("pair_D"),
                         pix=cache.export("pair_pix"), img=B.lm_render(x, sc.sh_degree, cams, ctx=ctx).cpu().numpy(),
                         u=u.cpu().numpy(), b=b.cpu().numpy(), M=M.cpu().numpy(), g=g.cpu().numpy(),
                         d=d[0].cpu().numpy(), fsq=float(fsq.item()))
        with pytest.raises(RuntimeError):
            ctx.destroy()                    # the cache is still alive
        cache.destroy()
    assert sum(used) > 0                      # the torch context's memory came from torch
    ctx_t.destroy()
    ctx_h.destroy()
    a, h = out["torch"], out["hip"]
    for k in ("vals", "T", "D", "pix", "img", "u"):
        np.testing.assert_array_equal(a[k], h[k], err_msg=k)
    assert a["fsq"] == h["fsq"]
    for k in ("b", "M", "g", "d"):
        assert rel(a[k], h[k]) <= 1e-6, k


def test_graph_mode_and_profiling_are_per_context():
    from paper_2409_12892_amd import binding as B
    pr = make_problem("tiny", with_J=False)
    sc, cams = pr["scene"], pr["cams"]
    x = torch.from_numpy(sc.x).cuda()
    tgt = torch.from_numpy(pr["target"].ravel()).cuda()
    c1, c2 = B.Ctx(), B.Ctx()
    B.lm_pcg_use_graph(1, ctx=c1)
    B.lm_pcg_use_graph(0, ctx=c2)
    B.lm_profile_enable(True, ctx=c1)
    res = {}
    for name, ctx in (("c1", c1), ("c2", c2)):
        cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt, ctx=ctx)
        M = B.lm_jacobi_diag(cache)
        d, st = B.lm_pcg_solve([cache], [b], [M], 1e-2, 6)
        res[name] = d[0].cpu().numpy()
        cache.destroy()
    p1 = B.lm_profile_read(ctx=c1)
    p2 = B.lm_profile_read(ctx=c2)
    B.lm_profile_enable(False, ctx=c1)
    assert "pcg_iteration_graph" in p1 and p1["pcg_iteration_graph"][0] == 6
    assert "apply_tile_JtJ" in p1
    assert p2 == {}
    assert rel(res["c1"], res["c2"]) <= 1e-5
    c1.destroy()
    c2.destroy()


def test_vec_dot_and_axpy():
    from paper_2409_12892_amd import binding as B
    rng = np.random.default_rng(4)
    for n in (0, 1, 1000, 3_000_001):
        a = rng.normal(size=n).astype(np.float32)
        b = rng.normal(size=n).astype(np.float32)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dot = float(B.lm_vec_dot(ta, tb).item())
        ref = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        assert dot == pytest.approx(ref, rel=1e-12, abs=1e-12)
        y = B.lm_vec_axpy(ta, tb, 0.375).cpu().numpy()
        np.testing.assert_array_equal(y, (a.astype(np.float64) + 0.375 * b.astype(np.float64)).astype(np.float32))
    # in place
    ta = torch.ones(10, device="cuda")
    B.lm_vec_axpy(ta, torch.full((10,), 2.0, device="cuda"), 0.5, out=ta)
    assert torch.all(ta == 2.0)


def test_mlp_fallback_returns_the_warning():
    from paper_2409_12892_amd import binding as B
    w = torch.zeros(B.MLP_PARAMS, device="cuda")
    f = torch.zeros((8, 5), device="cuda")
    f[0, 2] = float("nan")
    lib = B.load()
    s = torch.empty((3, 5), device="cuda")
    sc = torch.empty((3, 5), device="cuda")
    nf = torch.zeros(1, device="cuda", dtype=torch.int32)
    st = lib.lm_mlp_forward(B._ptr(w), B._ptr(f), B.c_int64(5), B.c_int32(3), B._ptr(s), B._ptr(sc), B._ptr(nf),
                            B._stream())
    assert st == B.LM_WARN_FALLBACK_JACOBI
    assert int(nf.item()) == 3            # one per output of the sample
    assert torch.all(sc[:, 2] == 1.0)
    f[0, 2] = 0.0
    st = lib.lm_mlp_forward(B._ptr(w), B._ptr(f), B.c_int64(5), B.c_int32(3), B._ptr(s), B._ptr(sc), B._ptr(nf),
                            B._stream())
    assert st == B.LM_OK
