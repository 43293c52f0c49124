"""FP64 CPU oracle for the 3DGS Levenberg-Marquardt / PCG hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything
in this package.  The product path (the HIP library and its Python binding)
never imports it, and this package never imports the product path; the two
share nothing but the seeded input arrays.

Contents (each function cites the passage of the paper it follows):

* ``sh``        real spherical-harmonics colour basis (paper section 3.1)
* ``forward``   projection, tile binning, alpha-blending (eq. alpha-blending)
* ``jacobian``  explicit per-pair Jacobian blocks and the products J p, J^T u,
                diag(J^T J), b = -J^T F (eq. backward-pass, apply-j, apply-jt,
                diag-jtj)
* ``solve``     Algorithm 1 (PCG) exactly as printed, dense normal-equation
                solve, and the subset combination (eq. combine-pcg)
* ``objective`` the paper's square-root L1 / SSIM residuals and their
                per-pixel weights and colour gradients (eq. gn-loss,
                supplement A.4)
* ``precond``   per-Gaussian blocks of J^T J, targets and features of the
                learned diagonal preconditioner, and its reference MLP

Arithmetic is float64 throughout; the only float32 steps are the ones that
decide integers (tile rectangles and depth-sort keys), taken in the same
precision as the kernels.
"""
