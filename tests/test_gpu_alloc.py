"""Caller-supplied device memory: with PyTorch's caching allocator installed,
the cache's buffers show up in torch's allocated memory, the products are
bit-identical to those of a cache on hipMalloc memory, and destroying the
cache gives the memory back."""
import numpy as np
import pytest

from gpu_common import random_direction
from paper_2409_12892_amd import scenegen as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_cache_memory_from_the_torch_allocator():
    from paper_2409_12892_amd import binding as B
    d = sg.config_scene("tiny", N=900, subsets=[(3, 64, 64)], seed=51, deg=1)
    sc, cams = d["scene"], d["cams"][0]
    x = torch.from_numpy(sc.x).cuda()
    tgt = B.lm_render(torch.from_numpy(d["x_star"]).cuda(), sc.sh_degree, cams)
    p = torch.from_numpy(random_direction(sc.P, sc.N, seed=52)).cuda()
    ref_cache, ref_b, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt)
    ref_M = B.lm_jacobi_diag(ref_cache)
    ref_g = B.lm_apply_JtJ(ref_cache, p, 1e-2, ref_M)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    B.use_torch_allocator(True)
    try:
        cache, b, _ = B.lm_build_cache(x, sc.sh_degree, cams, tgt)
        M = B.lm_jacobi_diag(cache)
        g = B.lm_apply_JtJ(cache, p, 1e-2, M)
        torch.cuda.synchronize()
        grown = torch.cuda.memory_allocated() - before
        assert grown >= cache.info()["device_bytes"]
        assert torch.equal(b, ref_b) and torch.equal(M, ref_M) and torch.equal(g, ref_g)
        held = torch.cuda.memory_allocated()
        cache.destroy()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= held - cache_bytes_floor(ref_cache)
    finally:
        B.use_torch_allocator(False)
    ref_cache.destroy()


def cache_bytes_floor(c):
    return c.info()["cache_bytes"]
