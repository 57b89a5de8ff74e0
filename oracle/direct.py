"""Dense direct solves used to pin the iterative oracle (Sec. 2.1.1: a
Cholesky factorisation of A + mu I and two triangular solves; Sec. 4.2:
forming and factoring the restricted matrix)."""
import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import kernels


def full_krr(X, y, kind, sigma, mu):
    """beta = (A + mu I)^{-1} y by dense Cholesky (eq. exact_eqn)."""
    A = kernels.block(X, X, kind, sigma)
    c = cho_factor(A + mu * np.eye(A.shape[0]))
    return cho_solve(c, np.asarray(y, dtype=np.float64))


def restricted_krr(M, b):
    """beta_hat = M^{-1} b for M = A(S,:)A(:,S) + H formed densely."""
    c = cho_factor(M)
    return cho_solve(c, b)
