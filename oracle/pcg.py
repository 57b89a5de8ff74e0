"""Textbook preconditioned conjugate gradient (Sec. 3, eq. psd_system;
Saad, Iterative Methods, Sec. 9.2), oracle side, FP64.

Zero initial iterate; stop when ||r|| / ||b|| <= tol on the recursive
residual.  Several right-hand sides are several independent recurrences;
a column that has converged is frozen.  At exit the true residual
||b - M x|| / ||b|| is computed with one explicit product.
"""
import numpy as np


def pcg(product, precond, b, tol, max_iter, history=None):
    """Solve M x = b.  ``product`` and ``precond`` map (n, m) -> (n, m).

    Returns (x, info) with info = dict(iters=per-column iterations,
    relres_recursive=..., relres_true=...).
    """
    b = np.asarray(b, dtype=np.float64)
    squeeze = b.ndim == 1
    B = b[:, None] if squeeze else b
    n, m = B.shape
    X = np.zeros_like(B)
    R = B.copy()
    bnorm = np.linalg.norm(B, axis=0)
    active = bnorm > 0
    iters = np.zeros(m, dtype=np.int64)
    Z = precond(R)
    P = Z.copy()
    rz = np.sum(R * Z, axis=0)
    it = 0
    while np.any(active) and it < max_iter:
        W = product(P)
        pw = np.sum(P * W, axis=0)
        alpha = np.where(active, rz / np.where(active, pw, 1.0), 0.0)
        X += alpha * P
        R -= alpha * W
        it += 1
        iters[active] = it
        rn = np.linalg.norm(R, axis=0)
        if history is not None:
            history.append(rn / np.where(bnorm > 0, bnorm, 1.0))
        active = active & (rn > tol * bnorm)
        if not np.any(active):
            break
        Z = precond(R)
        rz_new = np.sum(R * Z, axis=0)
        beta = np.where(active, rz_new / np.where(active, rz, 1.0), 0.0)
        P = np.where(active, Z + beta * P, 0.0)
        rz = np.where(active, rz_new, rz)
    safe = np.where(bnorm > 0, bnorm, 1.0)
    rec = np.linalg.norm(R, axis=0) / safe
    true = np.linalg.norm(B - product(X), axis=0) / safe
    info = dict(iters=iters, relres_recursive=rec, relres_true=true,
                converged=bool(np.all(rec <= tol)))
    return (X[:, 0] if squeeze else X), info
