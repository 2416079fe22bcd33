"""ORACLE (test infrastructure only): Jacobi-preconditioned conjugate gradients.

The paper solves its linear boundary value problems with a preconditioned
Krylov method (PETSc, Sec. 4).  Reading: k independent Jacobi-PCG recurrences,
one per right-hand side column, that share each matrix product; every column
has its own alpha and beta, starts from the supplied x0, and is frozen as
soon as its residual satisfies ||b_i - S x_i||_2 <= tol ||b_i||_2 (tested
before the first iteration and after every update).
"""
import numpy as np


def jacobi_pcg(S, B, X0=None, tol=1e-8, max_iter=10000):
    """Solve S X = B column by column.  S: scipy CSR (SPD), B: [N] or [N][k].
    Returns (X, iters[k], relres[k]) where relres uses the recursively
    updated residual."""
    vec = B.ndim == 1
    B2 = B.reshape(B.shape[0], -1).astype(np.float64)
    N, k = B2.shape
    X = np.zeros_like(B2) if X0 is None else X0.reshape(N, -1).astype(np.float64).copy()
    d = S.diagonal()
    if np.any(d <= 0.0):
        raise FloatingPointError("non-positive diagonal: Jacobi preconditioner undefined")
    bnorm = np.linalg.norm(B2, axis=0)
    R = B2 - S @ X
    Zp = R / d[:, None]
    P = Zp.copy()
    rz = np.sum(R * Zp, axis=0)
    iters = np.zeros(k, dtype=np.int64)
    active = np.linalg.norm(R, axis=0) > tol * bnorm
    active &= bnorm > 0.0
    for _ in range(max_iter):
        if not active.any():
            break
        Q = S @ P
        pq = np.sum(P * Q, axis=0)
        if np.any(active & ~(pq > 0.0)):
            raise FloatingPointError("PCG breakdown: p^T S p <= 0")
        alpha = np.where(active, rz / np.where(active, pq, 1.0), 0.0)
        X += alpha[None, :] * P
        R -= alpha[None, :] * Q
        Zp = R / d[:, None]
        rz_new = np.sum(R * Zp, axis=0)
        iters += active
        rn = np.linalg.norm(R, axis=0)
        beta = np.where(active, rz_new / np.where(active, rz, 1.0), 0.0)
        P = np.where(active[None, :], Zp + beta[None, :] * P, P)
        rz = np.where(active, rz_new, rz)
        active &= rn > tol * bnorm
    relres = np.linalg.norm(R, axis=0) / np.where(bnorm > 0, bnorm, 1.0)
    if vec:
        return X[:, 0], iters, relres
    return X, iters, relres
