"""Index ranges at scale: 64 views of 1280x720 over the batching workload's
scene (1.5M Gaussians, SH 3) binned into 8x8 tiles keep more than 2^32
tile keys (after the tiles below a splat's alpha threshold are left out).  The cache must not depend on that: the pair count and
b = -J^T F match the 8x32-tile build up to the binning difference of the
two tile shapes (a splat's pixels beyond its 3-sigma rectangle contribute
only where the rectangle reaches their tile; about 1e-4 of the pairs,
1e-3 of b)."""
import numpy as np
import pytest

from paper_2409_12892_amd import scenegen as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_more_than_2_32_tile_keys():
    from paper_2409_12892_amd import binding as B
    print("[gpu scale] batching scene, 64 views 1280x720", flush=True)
    d = sg.config_scene("batching", subsets=[(64, 1280, 720)])
    sc, cams = d["scene"], d["cams"][0]
    x = torch.from_numpy(sc.x).cuda()
    tgt = B.lm_render(torch.from_numpy(d["x_star"]).cuda(), sc.sh_degree, cams)
    out = {}
    for tile in [(8, 8), (8, 32)]:
        print(f"[gpu scale] build {tile[0]}x{tile[1]}", flush=True)
        c, b, fsq = B.lm_build_cache(x, sc.sh_degree, cams, tgt, tile=tile, cache_dtype="bf16", compact=True)
        out[tile] = (c.info(), b.double().cpu(), float(fsq.item()))
        c.destroy()
        torch.cuda.empty_cache()
    i8, b8, f8 = out[(8, 8)]
    i32, b32, f32 = out[(8, 32)]
    assert i8["n_keys"] > 2 ** 32
    assert abs(i8["n_pairs"] - i32["n_pairs"]) <= 1e-3 * i32["n_pairs"]
    assert abs(f8 - f32) <= 1e-3 * f32
    assert float((b8 - b32).norm() / b32.norm()) < 5e-3
