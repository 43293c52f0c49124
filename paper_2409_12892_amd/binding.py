"""ctypes binding of liblm3dgs.so (include/lm3dgs.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Device buffers are torch tensors on the current HIP device; the
work is enqueued on torch's current stream.  Importing this module does not
load the library; the first call does, and raises if it is missing (there is
no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblm3dgs.so")

LM_OK = 0
LM_WARN_BREAKDOWN = 1
LM_WARN_FALLBACK_JACOBI = 2
CACHE_DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
TOL_NONE, TOL_PAPER_SQUARED, TOL_RELATIVE = 0, 1, 2
PCG_MAX_HISTORY = 257

EXPORT = dict(records=0, sorted_values=1, tile_ranges=2, image=3, ncontrib=4, pair_T=5, pair_D=6,
              pair_pix=7, pair_gauss=8, residual=9, pair_flags=10, tile_segments=11)
_EXPORT_DTYPE = dict(records=np.float32, sorted_values=np.uint32, tile_ranges=np.int64, image=np.float32,
                     ncontrib=np.int32, pair_T=np.float32, pair_D=np.float32, pair_pix=np.int32,
                     pair_gauss=np.int32, residual=np.float32, pair_flags=np.int32, tile_segments=np.int64)

EXPORTED_SYMBOLS = (
    "lm_last_error", "lm_build_cache", "lm_cache_destroy", "lm_cache_get_info", "lm_jacobi_diag",
    "lm_apply_JtJ", "lm_apply_J", "lm_apply_JT", "lm_pcg_solve", "lm_combine_subsets", "lm_render",
    "lm_cache_export_size", "lm_cache_export", "lm_profile_enable", "lm_profile_read", "lm_residual_sqnorm",
    "lm_cache_view_sqnorm", "lm_pcg_use_graph", "lm_autotune_tile", "lm_pair_coverage", "lm_block_jacobi",
    "lm_precond_targets", "lm_precond_features", "lm_mlp_forward", "lm_mlp_workspace_bytes", "lm_mlp_train_step",
    "lm_jp_sqnorm", "lm_set_allocator", "lm_objective_terms", "lm_set_residual_weights", "lm_cache_objective",
    "lm_objective_value", "lm_pcg_solve_block", "lm_block_precond_apply", "lm_ctx_create", "lm_ctx_destroy",
    "lm_vec_dot", "lm_vec_axpy", "lm_vec_dot_static", "lm_cache_memory",
    "lm_cache_trim",
)

# objective kinds (include/lm3dgs.h): plain least squares, and the paper's
# square-root L1 / SSIM residuals with lambda1 = 0.8, lambda2 = 0.2
OBJ_L2, OBJ_L1_SSIM = 0, 1
OBJ_LAMBDA1, OBJ_LAMBDA2, OBJ_EPS = 0.8, 0.2, 1e-4

MLP_FEATURES, MLP_HIDDEN, MLP_MAX_OUT, MLP_PARAMS = 8, 64, 64, 8896
# offsets of the weight layout: W1 [8][64], b1, W2 [64][64], b2, W3 [64][64], b3
MLP_OFFSETS = dict(W1=(0, (8, 64)), b1=(512, (64,)), W2=(576, (64, 64)), b2=(4672, (64,)),
                   W3=(4736, (64, 64)), b3=(8832, (64,)))


class LmBufferBytes(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("bytes", ctypes.c_uint64)]


class LmObjective(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("lambda1", c_float), ("lambda2", c_float), ("eps", c_float)]


def objective(kind=OBJ_L1_SSIM, lambda1=OBJ_LAMBDA1, lambda2=OBJ_LAMBDA2, eps=OBJ_EPS) -> LmObjective:
    if isinstance(kind, str):
        kind = {"l2": OBJ_L2, "l1_ssim": OBJ_L1_SSIM}[kind]
    return LmObjective(int(kind), float(lambda1), float(lambda2), float(eps))


class LmCamera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("W", c_int32), ("H", c_int32)]


class LmScene(ctypes.Structure):
    _fields_ = [("N", c_int64), ("sh_degree", c_int32), ("reserved", c_int32), ("x", c_void_p)]


class LmOptions(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("cache_dtype", c_int32), ("flags", c_int32),
                ("scratch", c_void_p), ("ctx", c_void_p), ("thin_window", c_int32), ("reserved", c_int32)]


class Ctx:
    """Owner of one lm_ctx (its allocator, PCG launch mode and profiling
    records); allocator is an LmAllocator kept alive with the context, or
    None for hipMalloc."""

    def __init__(self, allocator=None):
        self.allocator = allocator
        h = c_void_p(0)
        _check(load().lm_ctx_create(byref(allocator) if allocator is not None else None, byref(h)), "lm_ctx_create")
        self.handle = h

    def destroy(self):
        if self.handle and self.handle.value:
            _check(load().lm_ctx_destroy(self.handle), "lm_ctx_destroy")
            self.handle = c_void_p(0)


def _ctx_ptr(ctx):
    # a c_void_p, not a Python int: ctypes passes a bare int as a 32-bit C int
    return None if ctx is None else c_void_p(ctx.handle.value)


def _opts(tile, cache_dtype=0, flags=0, ctx=None, thin_window=0):
    o = LmOptions(tile[0], tile[1], cache_dtype, flags)
    o.ctx = _ctx_ptr(ctx)
    o.thin_window = int(thin_window)
    return o


class LmCacheInfo(ctypes.Structure):
    _fields_ = [("N", c_int64), ("n_keys", c_int64), ("n_pairs", c_int64), ("n_segments", c_int64),
                ("n_gv", c_int64), ("n_pixels", c_int64), ("n_tiles", c_int64), ("n_pair_slots", c_int64),
                ("cache_bytes", c_int64),
                ("device_bytes", c_int64), ("V", c_int32), ("P", c_int32), ("tile_w", c_int32),
                ("tile_h", c_int32), ("cache_dtype", c_int32), ("sh_degree", c_int32),
                ("thin_window", c_int32), ("reserved", c_int32), ("n_pieces", c_int64),
                ("n_checkpoints", c_int64)]


class LmTileScore(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("build_ms", c_float), ("apply_ms", c_float)]


class LmProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", c_int32), ("reserved", c_int32),
                ("total_ms", c_double)]


class LmPcgStats(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("b_sqnorm", c_double),
                ("history", c_double * PCG_MAX_HISTORY)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2409_12892_amd.build_lib` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    lib.lm_last_error.restype = ctypes.c_char_p
    lib.lm_cache_export_size.restype = c_int64
    lib.lm_mlp_workspace_bytes.restype = ctypes.c_size_t
    for name in EXPORTED_SYMBOLS:
        if name not in ("lm_last_error", "lm_cache_export_size", "lm_mlp_workspace_bytes"):
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def _check(status: int, what: str) -> int:
    if status < 0:
        msg = load().lm_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed with status {status}: {msg}")
    return status


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> c_void_p:
    return c_void_p(0 if t is None else t.data_ptr())


def _dev_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
    return t


def camera_array(cams) -> ctypes.Array:
    """ctypes array of lm_camera from a Cameras-like object (R, t, fx, fy, cx, cy, W, H arrays)."""
    V = int(cams.R.shape[0])
    arr = (LmCamera * V)()
    for v in range(V):
        c = arr[v]
        c.R[:] = [float(a) for a in np.asarray(cams.R[v], np.float32).reshape(9)]
        c.t[:] = [float(a) for a in np.asarray(cams.t[v], np.float32).reshape(3)]
        c.fx, c.fy = float(cams.fx[v]), float(cams.fy[v])
        c.cx, c.cy = float(cams.cx[v]), float(cams.cy[v])
        c.W, c.H = int(cams.W[v]), int(cams.H[v])
    return arr


class Cache:
    """Owner of one lm_cache handle (one image subset)."""

    def __init__(self):
        self.handle = c_void_p(0)
        self.N = self.P = self.V = 0

    def info(self) -> dict:
        inf = LmCacheInfo()
        _check(load().lm_cache_get_info(self.handle, byref(inf)), "lm_cache_get_info")
        return {f: getattr(inf, f) for f, _ in LmCacheInfo._fields_}

    def memory(self) -> dict:
        """Device bytes held per buffer (name -> bytes, nonzero entries)."""
        lib = load()
        n = c_int32(0)
        _check(lib.lm_cache_memory(self.handle, None, 0, byref(n)), "lm_cache_memory")
        out = (LmBufferBytes * n.value)()
        _check(lib.lm_cache_memory(self.handle, out, n, byref(n)), "lm_cache_memory")
        return {e.name.decode(): int(e.bytes) for e in out if e.bytes}

    def trim(self):
        """Free what the products and PCG do not read (recomputed on demand)."""
        _check(load().lm_cache_trim(self.handle, _stream()), "lm_cache_trim")

    def export(self, what: str) -> np.ndarray:
        lib = load()
        code = EXPORT[what]
        n = lib.lm_cache_export_size(self.handle, code)
        if n < 0:
            raise RuntimeError(f"lm_cache_export_size({what}) failed")
        out = np.empty(n // np.dtype(_EXPORT_DTYPE[what]).itemsize, _EXPORT_DTYPE[what])
        _check(lib.lm_cache_export(self.handle, code, out.ctypes.data_as(c_void_p), c_int64(n), _stream()),
               "lm_cache_export")
        return out

    def destroy(self):
        if self.handle and self.handle.value:
            load().lm_cache_destroy(self.handle)
            self.handle = c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


BUILD_COMPACT = 1


def lm_build_cache(x, sh_degree: int, cams, target, *, tile=(16, 16), cache_dtype: str = "f32",
                   cache: Cache | None = None, want_b: bool = True, b=None, compact: bool = False,
                   scratch: Cache | None = None, ctx: Ctx | None = None, thin_window: int = 0):
    """Build the gradient cache of one subset.  Returns (cache, b, F_sqnorm)
    with b = -J^T F as a [P, N] tensor (written into `b` when given) and
    ||F||^2 as a 1-element float64 tensor (both None when want_b is False).
    With compact=True and a `scratch` Cache (possibly empty), the build's
    transient buffers are kept in `scratch` for the next compact build.
    thin_window=K > 0 builds the thinned cache (blend state of every K-th
    contributor per pixel; the products re-blend the pairs)."""
    import torch
    lib = load()
    x = _dev_f32(x, "x")
    target = _dev_f32(target, "target")
    P, N = x.shape
    scene = LmScene(N, sh_degree, 0, x.data_ptr())
    opts = _opts(tile, CACHE_DTYPES[cache_dtype], BUILD_COMPACT if compact else 0, ctx, thin_window)
    sh = None
    if scratch is not None:
        if not compact:
            raise ValueError("a scratch handle serves compact builds only")
        sh = c_void_p(scratch.handle.value)
        opts.scratch = ctypes.cast(ctypes.pointer(sh), c_void_p)
    carr = camera_array(cams)
    cache = Cache() if cache is None else cache
    if want_b and b is None:
        b = torch.empty((P, N), device=x.device, dtype=torch.float32)
    elif not want_b:
        b = None
    fsq = torch.empty(1, device=x.device, dtype=torch.float64) if want_b else None
    h = cache.handle
    try:
        _check(lib.lm_build_cache(byref(scene), carr, c_int32(len(carr)), _ptr(target), byref(opts), _stream(),
                                  byref(h), _ptr(b), _ptr(fsq)), "lm_build_cache")
    finally:
        if sh is not None:
            scratch.handle = sh
    cache.handle = h
    cache.N, cache.P, cache.V = N, P, len(carr)
    return cache, b, fsq


def lm_jacobi_diag(cache: Cache, out=None):
    import torch
    out = torch.empty((cache.P, cache.N), device="cuda", dtype=torch.float32) if out is None else out
    _check(load().lm_jacobi_diag(cache.handle, _ptr(out), _stream()), "lm_jacobi_diag")
    return out


def lm_apply_JtJ(cache: Cache, p, lam: float = 0.0, M=None, out=None, want_jp_sqnorm: bool = False):
    import torch
    p = _dev_f32(p, "p")
    out = torch.empty_like(p) if out is None else out
    jp = torch.empty(1, device=p.device, dtype=torch.float64) if want_jp_sqnorm else None
    _check(load().lm_apply_JtJ(cache.handle, _ptr(p), c_float(lam), _ptr(M), _ptr(out), _ptr(jp), _stream()),
           "lm_apply_JtJ")
    return (out, jp) if want_jp_sqnorm else out


def lm_apply_J(cache: Cache, p, out=None, n_residuals: int | None = None):
    import torch
    p = _dev_f32(p, "p")
    if out is None:
        n = n_residuals if n_residuals is not None else 3 * cache.info()["n_pixels"]
        out = torch.empty(n, device=p.device, dtype=torch.float32)
    _check(load().lm_apply_J(cache.handle, _ptr(p), _ptr(out), _stream()), "lm_apply_J")
    return out


class LmAllocator(ctypes.Structure):
    _fields_ = [("user", c_void_p),
                ("alloc", ctypes.CFUNCTYPE(c_void_p, c_void_p, ctypes.c_size_t, c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p))]


_torch_allocator = None


def use_torch_allocator(on: bool = True) -> None:
    """Route the library's device memory through PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / _delete on the call's stream), or
    back to hipMalloc / hipFree."""
    global _torch_allocator
    if not on:
        _check(load().lm_set_allocator(None), "lm_set_allocator")
        return
    import torch

    def _alloc(user, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
        except Exception:   # an exception cannot cross the C boundary: report NULL
            return None

    def _free(user, ptr, stream):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    a = LmAllocator(None, LmAllocator._fields_[1][1](_alloc), LmAllocator._fields_[2][1](_free))
    _torch_allocator = a        # the callbacks must outlive every buffer they allocated
    _check(load().lm_set_allocator(byref(a)), "lm_set_allocator")


def lm_jp_sqnorm(cache: Cache, p):
    """||J p||^2 as a 1-element float64 device tensor."""
    import torch
    p = _dev_f32(p, "p")
    out = torch.empty(1, device=p.device, dtype=torch.float64)
    _check(load().lm_jp_sqnorm(cache.handle, _ptr(p), _ptr(out), _stream()), "lm_jp_sqnorm")
    return out


def lm_apply_JT(cache: Cache, u, out=None):
    import torch
    u = _dev_f32(u, "u")
    out = torch.empty((cache.P, cache.N), device=u.device, dtype=torch.float32) if out is None else out
    _check(load().lm_apply_JT(cache.handle, _ptr(u), _ptr(out), _stream()), "lm_apply_JT")
    return out


def lm_pcg_solve(caches, bs, Ms, lam: float, n_iters: int, tol: float = 0.0, tol_mode: int = TOL_NONE,
                 scales=None, deltas=None, diag_floor: float = 0.0, block: bool = False):
    """Algorithm 1 for each subset; returns (deltas, stats dicts).  diag_floor
    = 0 is Algorithm 1 exactly (see lm_pcg_solve in include/lm3dgs.h);
    block=True uses the block-Jacobi preconditioner (lm_pcg_solve_block)."""
    import torch
    nb = len(caches)
    deltas = [torch.empty_like(b) for b in bs] if deltas is None else deltas
    H = (c_void_p * nb)(*[c.handle for c in caches])
    B = (c_void_p * nb)(*[b.data_ptr() for b in bs])
    Mm = (c_void_p * nb)(*[m.data_ptr() for m in Ms])
    D = (c_void_p * nb)(*[d.data_ptr() for d in deltas])
    Sc = None if scales is None else (c_void_p * nb)(*[0 if s is None else s.data_ptr() for s in scales])
    stats = (LmPcgStats * nb)()
    if block:
        if scales is not None:
            raise ValueError("the block-Jacobi solve takes no diagonal scaling")
        _check(load().lm_pcg_solve_block(H, c_int32(nb), B, Mm, c_float(lam), c_float(diag_floor), c_int32(n_iters),
                                         c_double(tol), c_int32(tol_mode), D, stats, _stream()), "lm_pcg_solve_block")
    else:
        _check(load().lm_pcg_solve(H, c_int32(nb), B, Mm, c_float(lam), c_float(diag_floor), c_int32(n_iters),
                                   c_double(tol),
                                   c_int32(tol_mode), Sc, D, stats, _stream()), "lm_pcg_solve")
    out = [dict(iters=s.iters, status=s.status, b_sqnorm=s.b_sqnorm,
                history=np.array(s.history[:s.iters + 1])) for s in stats]
    return deltas, out


def lm_block_precond_apply(cache: Cache, r, lam: float, diag_floor: float = 0.0, out=None,
                           count_fallback: bool = False):
    """z = A^-1 r with the cache's block-Jacobi factors for (lam, diag_floor);
    returns z, or (z, number of Gaussians that fell back to their damped
    diagonal) with count_fallback."""
    import torch
    r = _dev_f32(r, "r")
    out = torch.empty_like(r) if out is None else out
    nf = c_int32(0)
    _check(load().lm_block_precond_apply(cache.handle, c_float(lam), c_float(diag_floor), _ptr(r), _ptr(out),
                                         byref(nf) if count_fallback else None, _stream()), "lm_block_precond_apply")
    return (out, int(nf.value)) if count_fallback else out


def lm_combine_subsets(deltas, Ms, out=None):
    import torch
    nb = len(deltas)
    out = torch.empty_like(deltas[0]) if out is None else out
    D = (c_void_p * nb)(*[d.data_ptr() for d in deltas])
    Mm = (c_void_p * nb)(*[m.data_ptr() for m in Ms])
    _check(load().lm_combine_subsets(c_int32(nb), D, Mm, c_int64(deltas[0].numel()), _ptr(out), _stream()),
           "lm_combine_subsets")
    return out


def lm_residual_sqnorm(x, sh_degree: int, cams, target, *, tile=(16, 16), workspace: Cache | None = None,
                       out=None, ctx: Ctx | None = None):
    """||render(x) - target||^2 over the views of `cams` (forward pass only).
    Returns (value as a 1-element float64 device tensor, workspace)."""
    import torch
    x = _dev_f32(x, "x")
    target = _dev_f32(target, "target")
    P, N = x.shape
    scene = LmScene(N, sh_degree, 0, x.data_ptr())
    opts = _opts(tile, ctx=ctx)
    carr = camera_array(cams)
    ws = Cache() if workspace is None else workspace
    out = torch.empty(1, device=x.device, dtype=torch.float64) if out is None else out
    h = ws.handle
    _check(load().lm_residual_sqnorm(byref(scene), carr, c_int32(len(carr)), _ptr(target), byref(opts), _stream(),
                                     byref(h), _ptr(out)), "lm_residual_sqnorm")
    ws.handle = h
    return out, ws


def lm_objective_terms(image, target, cams, obj: LmObjective, *, w=True, e=True, workspace: Cache | None = None):
    """Objective terms of device images [V][3][H][W] (flattened): returns
    (w or None, e or None, E as a 1-element float64 device tensor, workspace)."""
    import torch
    image = _dev_f32(image, "image")
    target = _dev_f32(target, "target")
    carr = camera_array(cams)
    ws = Cache() if workspace is None else workspace
    wt = torch.empty_like(image) if w is True else (w if w is not False else None)
    et = torch.empty_like(image) if e is True else (e if e is not False else None)
    E = torch.empty(1, device=image.device, dtype=torch.float64)
    h = ws.handle
    _check(load().lm_objective_terms(_ptr(image), _ptr(target), carr, c_int32(len(carr)), byref(obj), _ptr(wt),
                                     _ptr(et), _ptr(E), _stream(), byref(h)), "lm_objective_terms")
    ws.handle = h
    return wt, et, E, ws


def lm_set_residual_weights(cache: Cache, w=None):
    """Residual weights (image layout) for every later product of the cache;
    None returns to plain least squares."""
    _check(load().lm_set_residual_weights(cache.handle, _ptr(None if w is None else _dev_f32(w, "w")), _stream()),
           "lm_set_residual_weights")


def lm_cache_objective(cache: Cache, target, obj: LmObjective, *, b=None, want_b=True):
    """Objective at the cache's point: sets the residual weights and returns
    (b = -J^T e or None, per-view E as a float64 device tensor [V])."""
    import torch
    target = _dev_f32(target, "target")
    info = cache.info()
    if want_b and b is None:
        b = torch.empty((info["P"], info["N"]), device=target.device, dtype=torch.float32)
    E = torch.empty(info["V"], device=target.device, dtype=torch.float64)
    _check(load().lm_cache_objective(cache.handle, _ptr(target), byref(obj), _ptr(b if want_b else None), _ptr(E),
                                     _stream()), "lm_cache_objective")
    return (b if want_b else None), E


def lm_objective_value(x, sh_degree: int, cams, target, obj: LmObjective, *, tile=(16, 16),
                       workspace: Cache | None = None, out=None, ctx: Ctx | None = None):
    """Objective of a forward render over the views of `cams`.  Returns
    (value as a 1-element float64 device tensor, workspace)."""
    import torch
    x = _dev_f32(x, "x")
    target = _dev_f32(target, "target")
    P, N = x.shape
    scene = LmScene(N, sh_degree, 0, x.data_ptr())
    opts = _opts(tile, ctx=ctx)
    carr = camera_array(cams)
    ws = Cache() if workspace is None else workspace
    out = torch.empty(1, device=x.device, dtype=torch.float64) if out is None else out
    h = ws.handle
    _check(load().lm_objective_value(byref(scene), carr, c_int32(len(carr)), _ptr(target), byref(opts), byref(obj),
                                     _stream(), byref(h), _ptr(out)), "lm_objective_value")
    ws.handle = h
    return out, ws


def lm_cache_view_sqnorm(cache: Cache, out=None):
    """Per-view ||F||^2 of a built cache (float64 device tensor [V])."""
    import torch
    V = cache.info()["V"]
    out = torch.empty(V, device="cuda", dtype=torch.float64) if out is None else out
    _check(load().lm_cache_view_sqnorm(cache.handle, _ptr(out), _stream()), "lm_cache_view_sqnorm")
    return out


def lm_autotune_tile(x, sh_degree: int, cams, target, *, cache_dtype: str = "f32", n_products: int = 10,
                     ctx: Ctx | None = None, thin_window: int = 0):
    """Measured tile shape for one subset: ((tile_w, tile_h), [per-candidate
    dicts with build_ms and apply_ms])."""
    x = _dev_f32(x, "x")
    target = _dev_f32(target, "target")
    P, N = x.shape
    scene = LmScene(N, sh_degree, 0, x.data_ptr())
    carr = camera_array(cams)
    tw, th, ns = c_int32(0), c_int32(0), c_int32(0)
    sc = (LmTileScore * 16)()
    opts = _opts((0, 0), CACHE_DTYPES[cache_dtype], 0, ctx, thin_window)
    _check(load().lm_autotune_tile(byref(scene), carr, c_int32(len(carr)), _ptr(target), byref(opts),
                                   c_int32(n_products), _stream(), byref(tw), byref(th), sc, c_int32(16), byref(ns)),
           "lm_autotune_tile")
    return (tw.value, th.value), [dict(tile=(sc[i].tile_w, sc[i].tile_h), build_ms=sc[i].build_ms,
                                       apply_ms=sc[i].apply_ms) for i in range(ns.value)]


def lm_pcg_use_graph(mode: int, ctx: Ctx | None = None) -> None:
    """0: eager iterations, 1: graph replay, 2: graph replay for batches (default)."""
    _check(load().lm_pcg_use_graph(_ctx_ptr(ctx), c_int32(mode)), "lm_pcg_use_graph")


def lm_profile_enable(on: bool = True, ctx: Ctx | None = None) -> None:
    _check(load().lm_profile_enable(_ctx_ptr(ctx), c_int32(1 if on else 0)), "lm_profile_enable")


def lm_profile_read(ctx: Ctx | None = None) -> dict:
    """{kernel group: (launches, total ms)} recorded since the last read."""
    arr = (LmProfileEntry * 64)()
    n = load().lm_profile_read(_ctx_ptr(ctx), arr, c_int32(64))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n)}


def lm_vec_dot(a, b, out=None, ctx: Ctx | None = None):
    """a . b in float64 (1-element device tensor) for float32 device vectors."""
    import torch
    a = _dev_f32(a, "a")
    b = _dev_f32(b, "b")
    if a.numel() != b.numel():
        raise ValueError("lm_vec_dot: sizes differ")
    out = torch.empty(1, device=a.device, dtype=torch.float64) if out is None else out
    _check(load().lm_vec_dot(_ctx_ptr(ctx), _ptr(a), _ptr(b), c_int64(a.numel()), _ptr(out), _stream()),
           "lm_vec_dot")
    return out


def lm_vec_dot_static(a, b, out):
    """a . b in float64 into the caller's 1-element float64 device tensor
    `out`, with the library's static partial-sum array (allocates nothing)."""
    a = _dev_f32(a, "a")
    b = _dev_f32(b, "b")
    if a.numel() != b.numel():
        raise ValueError("lm_vec_dot_static: sizes differ")
    _check(load().lm_vec_dot_static(_ptr(a), _ptr(b), c_int64(a.numel()), _ptr(out), _stream()),
           "lm_vec_dot_static")
    return out


def lm_vec_axpy(x, d, gamma: float, out=None):
    """x + gamma d (float32 device tensors of one shape); out may be x."""
    import torch
    x = _dev_f32(x, "x")
    d = _dev_f32(d, "d")
    if x.numel() != d.numel():
        raise ValueError("lm_vec_axpy: sizes differ")
    out = torch.empty_like(x) if out is None else _dev_f32(out, "out")
    _check(load().lm_vec_axpy(_ptr(x), _ptr(d), c_float(gamma), c_int64(x.numel()), _ptr(out), _stream()),
           "lm_vec_axpy")
    return out


def lm_render(x, sh_degree: int, cams, *, tile=(16, 16), out=None, ctx: Ctx | None = None):
    """Forward render of every view into a flat float32 [V][3][H][W] tensor."""
    import torch
    x = _dev_f32(x, "x")
    P, N = x.shape
    carr = camera_array(cams)
    n = sum(3 * int(cams.W[v]) * int(cams.H[v]) for v in range(len(carr)))
    out = torch.empty(n, device=x.device, dtype=torch.float32) if out is None else out
    scene = LmScene(N, sh_degree, 0, x.data_ptr())
    opts = _opts(tile, ctx=ctx)
    _check(load().lm_render(byref(scene), carr, c_int32(len(carr)), byref(opts), _ptr(out), _stream()),
           "lm_render")
    return out


# ---- learned preconditioner -----------------------------------------------------

def lm_pair_coverage(cache: Cache, out=None):
    """Pairs per Gaussian over all views (float32 device tensor [N])."""
    import torch
    out = torch.empty(cache.N, device="cuda", dtype=torch.float32) if out is None else out
    _check(load().lm_pair_coverage(cache.handle, _ptr(out), _stream()), "lm_pair_coverage")
    return out


def lm_block_jacobi(cache: Cache, gaussians):
    """Dense J^T J blocks [n, P, P] of the listed Gaussians (int64 device tensor)."""
    import torch
    idx = gaussians
    if not (isinstance(idx, torch.Tensor) and idx.is_cuda and idx.dtype == torch.int64 and idx.is_contiguous()):
        raise TypeError("gaussians must be a contiguous int64 tensor on the GPU")
    if idx.numel() and (int(idx.min()) < 0 or int(idx.max()) >= cache.N):
        raise ValueError("gaussian index out of range")
    out = torch.empty((idx.numel(), cache.P, cache.P), device="cuda", dtype=torch.float32)
    _check(load().lm_block_jacobi(cache.handle, _ptr(idx), c_int64(idx.numel()), _ptr(out), _stream()),
           "lm_block_jacobi")
    return out


PRECOND_SHRINK = 0.5


def lm_precond_targets(cache: Cache, lam: float, diag_floor: float = 0.0, shrink: float = PRECOND_SHRINK):
    """(t, mask) float32 device tensors [P, N] (see lm_precond_targets in include/lm3dgs.h)."""
    import torch
    t = torch.empty((cache.P, cache.N), device="cuda", dtype=torch.float32)
    m = torch.empty_like(t)
    _check(load().lm_precond_targets(cache.handle, c_float(lam), c_float(diag_floor), c_float(shrink), _ptr(t),
                                     _ptr(m), _stream()), "lm_precond_targets")
    return t, m


def lm_precond_features(cache: Cache, x, M, out=None):
    """Features [8, N] from the parameters and the Jacobi diagonal."""
    import torch
    x = _dev_f32(x, "x")
    M = _dev_f32(M, "M")
    out = torch.empty((MLP_FEATURES, cache.N), device="cuda", dtype=torch.float32) if out is None else out
    _check(load().lm_precond_features(cache.handle, _ptr(x), _ptr(M), _ptr(out), _stream()), "lm_precond_features")
    return out


def mlp_init(p_out: int, seed: int = 0):
    """Float32 device weights [MLP_PARAMS]: normal W1 (std 1/sqrt(8)), W2 (1/8),
    W3 (0.1/8, columns >= p_out zero), zero biases."""
    import torch
    if not 1 <= p_out <= MLP_MAX_OUT:
        raise ValueError("p_out must be 1..64")
    gen = torch.Generator().manual_seed(seed)
    w = torch.zeros(MLP_PARAMS, dtype=torch.float32)
    for name, std in (("W1", MLP_FEATURES ** -0.5), ("W2", MLP_HIDDEN ** -0.5), ("W3", 0.1 * MLP_HIDDEN ** -0.5)):
        off, shape = MLP_OFFSETS[name]
        v = torch.randn(shape, generator=gen, dtype=torch.float32) * std
        if name == "W3":
            v[:, p_out:] = 0
        w[off:off + v.numel()] = v.reshape(-1)
    return w.cuda()


def mlp_unpack(w) -> dict:
    """Host float64 views of a weight vector by name (W1 [8, 64], ..., W3 [64, 64])."""
    a = w.detach().double().cpu().numpy() if hasattr(w, "detach") else np.asarray(w, np.float64)
    return {k: a[o:o + int(np.prod(sh))].reshape(sh) for k, (o, sh) in MLP_OFFSETS.items()}


def lm_mlp_forward(w, feat, p_out: int, want_s: bool = True, want_scale: bool = True):
    """(s, scale, n_fallback) for the columns of feat [8, n]."""
    import torch
    w = _dev_f32(w, "w")
    feat = _dev_f32(feat, "feat")
    n = feat.shape[1]
    s = torch.empty((p_out, n), device="cuda", dtype=torch.float32) if want_s else None
    sc = torch.empty((p_out, n), device="cuda", dtype=torch.float32) if want_scale else None
    nf = torch.zeros(1, device="cuda", dtype=torch.int32)
    _check(load().lm_mlp_forward(_ptr(w), _ptr(feat), c_int64(n), c_int32(p_out), _ptr(s), _ptr(sc), _ptr(nf),
                                 _stream()), "lm_mlp_forward")
    return s, sc, nf


class MlpTrainer:
    """Adam state and workspace for lm_mlp_train_step on one weight vector."""

    def __init__(self, w, lr: float = 1e-3):
        import torch
        self.w = _dev_f32(w, "w")
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.lr = lr
        self.step_count = 0
        nbytes = int(load().lm_mlp_workspace_bytes())
        self.ws = torch.empty(nbytes, device="cuda", dtype=torch.uint8)

    def step(self, feat, target, mask, lr: float | None = None, want_grad: bool = False):
        """One Adam step; returns (loss device tensor [1] float64, grad or None),
        both taken at the weights before the step.  lr = 0 computes them only."""
        import torch
        feat = _dev_f32(feat, "feat")
        target = _dev_f32(target, "target")
        mask = _dev_f32(mask, "mask")
        p_out, n = target.shape
        lr = self.lr if lr is None else lr
        if lr > 0:
            self.step_count += 1
        loss = torch.empty(1, device="cuda", dtype=torch.float64)
        grad = torch.empty_like(self.w) if want_grad else None
        _check(load().lm_mlp_train_step(_ptr(self.w), _ptr(self.m), _ptr(self.v), c_int32(max(self.step_count, 1)),
                                        c_float(lr), _ptr(feat), _ptr(target), _ptr(mask), c_int64(n),
                                        c_int32(p_out), _ptr(grad), _ptr(loss), _ptr(self.ws),
                                        ctypes.c_size_t(self.ws.numel()), _stream()), "lm_mlp_train_step")
        return loss, grad

