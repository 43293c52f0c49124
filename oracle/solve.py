"""Normal-equation solves in float64: Algorithm 1 (PCG), a dense reference
solve, and the subset combination.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

TOL_NONE = 0
TOL_PAPER_SQUARED = 1     # break if ||r||^2 < tol * ||b||^2  (Algorithm 1 as printed, tol = 0.01)
TOL_RELATIVE = 2          # break if ||r|| < tol * ||b||


def jacobi_inverse(M: np.ndarray) -> np.ndarray:
    """M^{-1} = 1 / diag(J^T J) (section 3.3), 0 where the diagonal is 0
    (a parameter no residual sees keeps a zero update)."""
    M = np.asarray(M, np.float64)
    out = np.zeros_like(M)
    pos = M > 0
    out[pos] = 1.0 / M[pos]
    return out


def pcg(apply_JtJ, b: np.ndarray, M: np.ndarray, lam: float, n_iters: int,
        tol: float = 0.0, tol_mode: int = TOL_NONE, precond_scale: np.ndarray | None = None,
        diag_floor: float = 0.0, precond=None) -> dict:
    """Algorithm 1, in the order printed:

        x0 = M^-1 b;  r0 = b - (J^T J x0 + lam M x0);  z0 = M^-1 r0;  p0 = z0
        for i in 0 .. n_iters-1:
            g = J^T J p + lam M p;  alpha = r^T z / p^T g
            x += alpha p;  r -= alpha g;  z = M^-1 r
            beta = r_new^T z_new / r^T z;  p = z + beta p
            break if ||r||^2 < tol ||b||^2

    ``apply_JtJ(p)`` returns J^T J p (without the damping term).  The loop
    runs n_iters times (n_iters + 1 products in total: with n_iters = 8 the
    paper's "up to 9" applications).  ``precond_scale`` multiplies M^-1
    element-wise (a learned diagonal rescaling); None means plain Jacobi.
    ``diag_floor`` > 0 (not in the paper's text; the minimum LM diagonal of
    CERES, whose LM variant the paper follows) replaces every positive
    diagonal entry below the floor by the floor, in the damping term and in
    M^-1 alike; 0 runs Algorithm 1 as printed.  ``precond(v)``, when given,
    replaces every application of M^-1 (a block preconditioner); the damping
    term still uses M.
    Returns x and the per-iteration ||r||^2 / ||b||^2 history.
    """
    b = np.asarray(b, np.float64).ravel()
    M = np.asarray(M, np.float64).ravel()
    if diag_floor > 0.0:
        M = np.where(M > 0.0, np.maximum(M, diag_floor), 0.0)
    Minv = jacobi_inverse(M)
    if precond_scale is not None:
        Minv = Minv * np.asarray(precond_scale, np.float64).ravel()
    bb = float(b @ b)

    def A(v):
        return apply_JtJ(v) + lam * M * v

    Pinv = (lambda v: Minv * v) if precond is None else precond
    x = Pinv(b)
    r = b - A(x)
    z = Pinv(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [float(r @ r) / bb if bb > 0 else 0.0]
    status = 0
    it = 0
    for it in range(1, n_iters + 1):
        g = A(p)
        pg = float(p @ g)
        if not np.isfinite(pg) or pg <= 0.0:
            status = 1          # breakdown: keep the current iterate
            it -= 1
            break
        alpha = rz / pg
        x = x + alpha * p
        r = r - alpha * g
        z = Pinv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz if rz != 0.0 else 0.0
        p = z + beta * p
        rz = rz_new
        rr = float(r @ r)
        hist.append(rr / bb if bb > 0 else 0.0)
        if tol_mode == TOL_PAPER_SQUARED and rr < tol * bb:
            break
        if tol_mode == TOL_RELATIVE and np.sqrt(rr) < tol * np.sqrt(bb):
            break
    return dict(x=x, iters=it, history=np.asarray(hist), status=status)


def block_jacobi(blocks: np.ndarray, lam: float, diag_floor: float = 0.0):
    """Block-Jacobi preconditioner of the damped normal equations: per
    Gaussian k the P x P block A_k = B_k + lam diag(D_k) of
    J^T J + lam diag(D) (eq. norm-eq restricted to the Gaussian's own
    parameters; B_k = J_k^T J_k, D = diag(J^T J) raised to diag_floor where
    positive and smaller), inverted exactly.  A parameter with a zero
    diagonal (no residual sees it) keeps a unit diagonal and no coupling, so
    its entry passes through unchanged (its residual entry is 0).
    ``blocks`` [N, P, P]; returns v -> A^-1 v on [P][N]-ordered vectors."""
    blocks = np.asarray(blocks, np.float64)
    N, P, _ = blocks.shape
    A = blocks.copy()
    for k in range(N):
        d = np.diag(blocks[k]).copy()
        obs = d > 0
        A[k][~obs, :] = 0.0
        A[k][:, ~obs] = 0.0
        A[k][np.diag_indices(P)] = np.where(obs, d + lam * np.maximum(d, diag_floor), 1.0)

    def apply(v):
        V = np.asarray(v, np.float64).reshape(P, N)
        out = np.empty_like(V)
        for k in range(N):
            out[:, k] = np.linalg.solve(A[k], V[:, k])
        return out.ravel()
    return apply


def dense_solve(JtJ: np.ndarray, b: np.ndarray, lam: float, diag_floor: float = 0.0) -> np.ndarray:
    """Solve (J^T J + lam D) delta = b on the observed parameters (eq. norm-eq,
    D = diag(J^T J), raised to diag_floor where it is positive and smaller);
    unobserved parameters (zero diagonal) get 0."""
    A = np.asarray(JtJ.toarray() if hasattr(JtJ, "toarray") else JtJ, np.float64)
    d = np.diag(A).copy()
    obs = d > 0
    out = np.zeros(A.shape[0])
    D = np.maximum(d[obs], diag_floor)
    As = A[np.ix_(obs, obs)] + lam * np.diag(D)
    out[obs] = np.linalg.solve(As, np.asarray(b, np.float64).ravel()[obs])
    return out


def combine_subsets(deltas: list[np.ndarray], Ms: list[np.ndarray]) -> np.ndarray:
    """eq. combine-pcg: delta = sum_i M_i delta_i / sum_k M_k element-wise,
    with M_i = diag(J_i^T J_i); a parameter with zero total weight gets 0
    (the printed denominator index 'k = 1..n' is read as k = 1..n_b)."""
    num = np.zeros_like(np.asarray(deltas[0], np.float64).ravel())
    den = np.zeros_like(num)
    for d, m in zip(deltas, Ms):
        m = np.asarray(m, np.float64).ravel()
        num += m * np.asarray(d, np.float64).ravel()
        den += m
    out = np.zeros_like(num)
    pos = den > 0
    out[pos] = num[pos] / den[pos]
    return out
