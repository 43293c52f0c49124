"""lm_vec_dot_static, the dot product that allocates nothing, against
lm_vec_dot through the C ABI: two calls in a row on the library's static
partial-sum array, the second with a smaller input, each bit-identical to
lm_vec_dot (same kernels, same fixed grid, same summation order) and within
float64 rounding of the exact dot product of the float32 inputs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _exact(a, b):
    # float64 products of float32 values are exact; math.fsum rounds the sum once
    import math
    return math.fsum((a.astype(np.float64) * b.astype(np.float64)).tolist())


@pytest.mark.parametrize("sizes", [(3_000_001, 1_000), (700_000, 64), (5, 1)])
def test_vec_dot_static_matches_vec_dot(sizes):
    from paper_2409_12892_amd import binding as B
    gen = torch.Generator(device="cpu").manual_seed(sum(sizes))
    out_static = torch.full((1,), float("nan"), device="cuda", dtype=torch.float64)
    for n in sizes:
        a = torch.randn(n, generator=gen).cuda()
        b = torch.randn(n, generator=gen).cuda()
        B.lm_vec_dot_static(a, b, out_static)
        ref = B.lm_vec_dot(a, b)
        torch.cuda.synchronize()
        got, want = float(out_static.item()), float(ref.item())
        assert got == want, (n, got, want)
        exact = _exact(a.cpu().numpy(), b.cpu().numpy())
        scale = float(torch.dot(a.double().abs(), b.double().abs()).item())
        assert abs(got - exact) <= 1e-12 * max(scale, 1e-300), (n, got, exact)


def test_vec_dot_static_rejects_bad_sizes():
    import ctypes
    from paper_2409_12892_amd import binding as B
    lib = B.load()
    a = torch.ones(4, device="cuda")
    out = torch.zeros(1, device="cuda", dtype=torch.float64)
    st = lib.lm_vec_dot_static(B._ptr(a), B._ptr(a), ctypes.c_int64((1 << 40) + 1), B._ptr(out), B._stream())
    assert st == -3   # LM_ERR_CAPACITY, before any launch
    st = lib.lm_vec_dot_static(B._ptr(a), B._ptr(a), ctypes.c_int64(-1), B._ptr(out), B._stream())
    assert st == -1   # LM_ERR_INVALID_ARG
