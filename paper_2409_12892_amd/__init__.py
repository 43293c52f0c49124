"""MI355X (gfx950) hot path of the Levenberg-Marquardt optimiser for 3D
Gaussian Splatting (arXiv 2409.12892): gradient-cache build, J p / J^T u,
Jacobi preconditioner, PCG and subset combination, in HIP behind the C ABI
of include/lm3dgs.h.

Submodules: ``binding`` (ctypes calls into liblm3dgs.so, no CPU fallback),
``scenegen`` (seeded synthetic inputs), ``build_lib`` (hipcc build).
"""
__all__ = ["binding", "scenegen", "build_lib"]
