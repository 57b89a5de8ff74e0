"""The oracle's pins catch plausible mistakes: each test plants one mistake
in the oracle (a dropped term, a wrong sign or index, a transposed operand,
a wrong constant) and checks that the pin it should trip fails."""
import numpy as np
import pytest

import oracle.kernels as K
import oracle.rpcholesky as RP
import oracle.pcg as PCG
import oracle.krill as KR
from oracle import direct
import tests.test_oracle_kernels as TK
import tests.test_oracle_rpcholesky as TR
import tests.test_oracle_pcg as TP
import tests.test_oracle_krill as TKR
import tests.test_oracle_pivot_rules as TPR


def must_fail(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_gaussian_bandwidth_mistake_is_caught(monkeypatch):
    orig = K.block

    def bad(Xr, Xc, kind, sigma):  # sigma^2 instead of 2 sigma^2
        if kind == K.GAUSSIAN:
            return orig(Xr, Xc, kind, sigma / np.sqrt(2.0))
        return orig(Xr, Xc, kind, sigma)
    monkeypatch.setattr(K, "block", bad)
    must_fail(TK.test_block_matches_brute_force, K.GAUSSIAN)


def test_laplace_squared_distance_mistake_is_caught(monkeypatch):
    orig = K.block

    def bad(Xr, Xc, kind, sigma):  # l2 instead of l1
        if kind == K.LAPLACE:
            d2 = -2 * sigma * sigma * np.log(orig(Xr, Xc, K.GAUSSIAN, sigma))
            return np.exp(-np.sqrt(np.maximum(d2, 0)) / sigma)
        return orig(Xr, Xc, kind, sigma)
    monkeypatch.setattr(K, "block", bad)
    must_fail(TK.test_separable_product_form, K.LAPLACE)


def test_wrong_factor_update_is_caught(monkeypatch):
    orig = RP.rpcholesky

    def bad_rpchol(X, kind, sigma, r, B=None, seed=0, record=None):
        F, piv = orig(X, kind, sigma, r, B, seed, record)
        F[:, 1:] *= 1.01  # later columns updated wrongly
        return F, piv
    monkeypatch.setattr(RP, "rpcholesky", bad_rpchol)
    must_fail(TR.test_nystrom_identity_psd_residual_and_monotone_trace, K.GAUSSIAN)


def test_off_by_one_sampler_is_caught(monkeypatch):
    orig = RP.sample_index

    def bad(d, O, u):  # returns the neighbour of the correct index
        i = orig(d, O, u)
        return min(i + 1, len(d) - 1)
    monkeypatch.setattr(RP, "sample_index", bad)
    must_fail(TR.test_sampler_distribution_is_proportional_to_d)


def test_greedy_smallest_diagonal_mistake_is_caught(monkeypatch):
    orig = RP.select_block

    def bad(rule, d, pool, seed, b, count):  # smallest positive residual instead
        if rule == "greedy":
            return [int(np.argmin(np.where(d > 0, d, np.inf)))]
        return orig(rule, d, pool, seed, b, count)
    monkeypatch.setattr(RP, "select_block", bad)
    must_fail(TPR.test_greedy_trap_greedy_takes_the_identity_block_first)
    must_fail(TPR.test_greedy_equals_diagonal_pivoting, K.GAUSSIAN)


def test_uniform_weighted_by_residual_mistake_is_caught(monkeypatch):
    orig = RP.select_block

    def bad(rule, d, pool, seed, b, count):  # weights from d: RPCholesky again
        return orig("rpcholesky" if rule == "uniform" else rule, d, pool, seed, b, count)
    monkeypatch.setattr(RP, "select_block", bad)
    must_fail(TPR.test_rank2_block_uniform_misses_the_small_block_hypergeometrically)


def test_uniform_with_replacement_mistake_is_caught(monkeypatch):
    orig = RP.select_block

    def bad(rule, d, pool, seed, b, count):  # drawn indices not retired
        return orig(rule, d, np.ones_like(pool), seed, b, count)
    monkeypatch.setattr(RP, "select_block", bad)
    must_fail(TPR.test_uniform_blocks_budget_distinct_draws)


def test_transposed_triangular_solve_is_caught(monkeypatch):
    def bad_apply(self, Z):
        Z = np.asarray(Z, dtype=np.float64)
        squeeze = Z.ndim == 1
        Z2 = Z[:, None] if squeeze else Z
        coef = 1.0 / (self.s2 + self.mu) + 1.0 / self.mu  # wrong sign
        out = self.U @ (coef[:, None] * (self.U.T @ Z2)) + Z2 / self.mu
        return out[:, 0] if squeeze else out
    monkeypatch.setattr(RP.NystromPreconditioner, "apply", bad_apply)
    must_fail(TR.test_preconditioner_forms_agree_and_bounds_hold)


def test_wrong_pcg_sign_is_caught(monkeypatch):
    orig = PCG.pcg

    def bad(product, precond, b, tol, max_iter, history=None):
        x, info = orig(product, precond, b, tol, max_iter, history)
        return -x, info
    monkeypatch.setattr(PCG, "pcg", bad)
    must_fail(TP.test_rpcholesky_pcg_matches_dense_cholesky_solve)


def test_wrong_restricted_block_in_product_is_caught(monkeypatch):
    orig_init = KR.Krill.__init__

    def bad_init(self, *a, **kw):
        orig_init(self, *a, **kw)
        self.AnS = self.AnS + 1e-3  # a wrong A(:,S) in the product
    monkeypatch.setattr(KR.Krill, "__init__", bad_init)
    must_fail(TKR.test_all_points_as_centres_reduce_to_full_data_krr)


def _plant_shift(monkeypatch, bad_shift):
    """Replaces the diagonal shift of H (Alg. 2, step 2) by bad_shift(N, k, tr(A_SS))."""
    orig_init = KR.Krill.__init__

    def bad_init(self, *a, **kw):
        orig_init(self, *a, **kw)
        trace = float(np.trace(K.block(self.X[self.S], self.X[self.S], self.kind, self.sigma)))
        wrong = bad_shift(self.N, self.k, trace)
        self.H = self.H + (wrong - self.shift) * np.eye(self.k)
        self.P = self.B.T @ self.B + self.H
        try:
            self.C = np.linalg.cholesky(self.P).T
        except np.linalg.LinAlgError:  # without the shift P can be singular here
            self.C = None
    monkeypatch.setattr(KR.Krill, "__init__", bad_init)


@pytest.mark.parametrize("name,bad", [
    ("shift left out", lambda N, k, tr: 0.0),
    ("N dropped", lambda N, k, tr: KR.EPS * tr),
    ("trace over all N points", lambda N, k, tr: N * KR.EPS * N),
    ("squared trace", lambda N, k, tr: N * KR.EPS * tr * tr),
])
def test_krill_shift_mistakes_are_caught(monkeypatch, name, bad):
    _plant_shift(monkeypatch, bad)
    must_fail(TKR.test_krill_shift_on_singular_centres)


def test_single_precision_eps_in_krill_shift_is_caught(monkeypatch):
    monkeypatch.setattr(KR, "EPS", 2.0 ** -23)
    must_fail(TKR.test_krill_shift_on_singular_centres)


def test_krill_without_sketch_term_is_caught(monkeypatch):
    orig_init = KR.Krill.__init__

    def bad_init(self, *a, **kw):  # P = H: the B^T B term forgotten
        orig_init(self, *a, **kw)
        self.P = self.H.copy()
        self.C = np.linalg.cholesky(self.P).T
    monkeypatch.setattr(KR.Krill, "__init__", bad_init)
    must_fail(TKR.test_krill_kappa_on_a_restricted_system_as_mu_vanishes)


def test_wrong_sketch_scale_is_caught(monkeypatch):
    orig = KR.sketch_matrix

    def bad(N, d_rows, zeta, seed):
        return orig(N, d_rows, zeta, seed) * np.sqrt(zeta)  # forgot zeta^{-1/2}
    monkeypatch.setattr(KR, "sketch_matrix", bad)
    must_fail(TKR.test_sketch_structure)


def test_wrong_centre_indexing_in_prediction_is_caught(monkeypatch):
    import oracle.predict as PR
    import tests.test_oracle_predict as TPR

    def bad(X, S, beta_hat, Xtest, kind, sigma, row_block=2048):  # off-by-one centres
        C = np.asarray(X)[(np.asarray(S) + 1) % len(X)]
        return K.matvec(Xtest, C, beta_hat, kind, sigma, row_block=row_block)
    monkeypatch.setattr(PR, "predict_restricted", bad)
    must_fail(TPR.test_restricted_fit_satisfies_the_normal_equations)


def test_smape_without_halving_is_caught(monkeypatch):
    import oracle.predict as PR
    import tests.test_oracle_predict as TPR

    def bad(yhat, y):  # denominator |yhat| + |y| (no halving)
        yhat = np.asarray(yhat, float)
        y = np.asarray(y, float)
        den = np.abs(yhat) + np.abs(y)
        return float(np.mean(np.divide(np.abs(yhat - y), den, out=np.zeros_like(den),
                                       where=den > 0)))
    monkeypatch.setattr(PR, "smape", bad)
    must_fail(TPR.test_smape_definition_values)
