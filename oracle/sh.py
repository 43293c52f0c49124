"""Real spherical-harmonics colour basis, degrees 0..3.

Paper section 3.1: the view-dependent colour of each Gaussian is a
spherical-harmonics expansion of order 3.  The paper does not print the
basis; this is the standard real basis (no Condon-Shortley phase), indexed
k = l*l + (m + l) for m = -l..l, evaluated at a unit direction d = (x, y, z).
Written with plain polynomials so that complex-step differentiation works.

Pinned in tests against scipy's complex spherical harmonics.
"""
import numpy as np

_C0 = 0.28209479177387814    # 1 / (2 sqrt(pi))
_C1 = 0.4886025119029199     # sqrt(3 / (4 pi))
_C2 = (1.0925484305920792, 1.0925484305920792, 0.31539156525252005,
       1.0925484305920792, 0.5462742152960396)
_C3 = (0.5900435899266435, 2.890611442640554, 0.4570457994644658,
       0.3731763325901154, 0.4570457994644658, 1.445305721320277,
       0.5900435899266435)


def sh_basis(d: np.ndarray, deg: int) -> np.ndarray:
    """Basis values Y_k(d), shape [(deg+1)^2, ...] for d of shape [3, ...].

    d must be a unit vector (the degree-2 and -3 polynomials use
    x^2 + y^2 + z^2 = 1 implicitly)."""
    x, y, z = d[0], d[1], d[2]
    out = [np.ones_like(x) * _C0]
    if deg >= 1:
        out += [_C1 * y, _C1 * z, _C1 * x]
    if deg >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [_C2[0] * x * y,
                _C2[1] * y * z,
                _C2[2] * (2.0 * zz - xx - yy),
                _C2[3] * x * z,
                _C2[4] * (xx - yy)]
    if deg >= 3:
        out += [_C3[0] * y * (3.0 * xx - yy),
                _C3[1] * x * y * z,
                _C3[2] * y * (4.0 * zz - xx - yy),
                _C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                _C3[4] * x * (4.0 * zz - xx - yy),
                _C3[5] * z * (xx - yy),
                _C3[6] * x * (xx - 3.0 * yy)]
    return np.stack(out)
