"""Out-of-sample prediction and its error measure (oracle side).

* ``predict_full``: the prediction function of full-data KRR (Sec. 2),
  f(x) = sum_i beta_i K(x_i, x) over the N training points.
* ``predict_restricted``: the prediction function of restricted KRR
  (Sec. 2.2), f(x) = sum_i beta_i K(x_{s_i}, x) over the k centres.
* ``smape``: the symmetric mean absolute percentage error used for the HOMO
  energy task (Sec. 4.1): the mean over test points of
  |yhat_i - y_i| / ((|yhat_i| + |y_i|) / 2).

Each prediction is the definition written out: a dense kernel block between
the test points and the expansion points, times the coefficients, in FP64.
"""
import numpy as np

from . import kernels


def predict_full(X, beta, Xtest, kind, sigma, row_block=2048):
    """f(Xtest) = K(Xtest, X) beta (Sec. 2); beta is N or N x m."""
    return kernels.matvec(Xtest, X, beta, kind, sigma, row_block=row_block)


def predict_restricted(X, S, beta_hat, Xtest, kind, sigma, row_block=2048):
    """f(Xtest) = K(Xtest, X(S,:)) beta_hat (Sec. 2.2); beta_hat is k or k x m."""
    C = np.asarray(X, dtype=np.float64)[np.asarray(S, dtype=np.int64)]
    return kernels.matvec(Xtest, C, beta_hat, kind, sigma, row_block=row_block)


def smape(yhat, y):
    """Symmetric mean absolute percentage error (Sec. 4.1).  A pair with
    yhat_i = y_i = 0 contributes 0 (the ratio's limit along yhat = y)."""
    yhat = np.asarray(yhat, dtype=np.float64).reshape(-1)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    den = (np.abs(yhat) + np.abs(y)) / 2.0
    num = np.abs(yhat - y)
    ratio = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
    return float(np.mean(ratio))
