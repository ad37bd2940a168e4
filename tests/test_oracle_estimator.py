"""Pins for oracle.estimator: Lemma 3 / Eq. (4), Eq. (13), Eq. (14) and the reduced test."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import estimator, pca
from paper_2411_17229_amd import workloads


@pytest.fixture(scope="module")
def small():
    X, _ = workloads.make_mixture(200, 16, 4, 1.2, 1, seed=1)
    mu, W, lam = pca.fit(X)
    return X.astype(np.float64), mu, W, lam


def test_order_statistic_by_hand():
    v = np.arange(10, 0, -1, dtype=float)          # 10..1
    assert estimator.order_statistic(v, 0.9) == 9.0  # ceil(9.0) = 9th smallest
    assert estimator.order_statistic(v, 0.95) == 10.0  # ceil(9.5) = 10th
    assert estimator.order_statistic(v, 0.01) == 1.0
    assert estimator.order_statistic_index(0.9, 100000) == 90000


def test_scale_by_hand():
    c = estimator.scale([4.0, 3.0, 2.0, 1.0])
    np.testing.assert_allclose(c, [2.5, 10 / 7, 10 / 9, 1.0], rtol=1e-15)


def test_p6_lemma3_unbiased_over_all_ordered_pairs(small):
    """Mean over all N^2 ordered pairs of c_d * ||W_d^T (x_i - x_j)||^2 = mean ||x_i - x_j||^2."""
    X, mu, W, lam = small
    Y = pca.rotate(X, mu, W)
    c = estimator.scale(lam)
    diff = Y[:, None, :] - Y[None, :, :]
    S = np.cumsum(diff ** 2, axis=2).reshape(-1, Y.shape[1])
    exact = np.mean(np.sum((X[:, None, :] - X[None, :, :]) ** 2, axis=2))
    est = c * S.mean(axis=0)
    assert np.max(np.abs(est - exact) / exact) <= 1e-12


def test_p7_estimate_at_full_dimension_is_exact(small):
    X, mu, W, lam = small
    Y = pca.rotate(X, mu, W)
    c = estimator.scale(lam)
    assert c[-1] == 1.0
    for i, j in [(0, 1), (5, 77), (10, 199)]:
        S_D = np.sum((Y[i] - Y[j]) ** 2)
        dis = math.sqrt(np.sum((X[i] - X[j]) ** 2))
        assert abs(float(estimator.estimate(S_D, c[-1])) - dis) / dis <= 1e-12


def test_p8_threshold_shape():
    X, _ = workloads.make_mixture(3000, 32, 8, 1.2, 1, seed=2)
    mu, W, lam = pca.fit(X)
    pairs = workloads.calibration_pairs(len(X), 20000, seed=2)
    eps, T, M = estimator.calibrate(X, W, lam, pairs, 0.1)
    assert M == 20000
    assert T[-1] == 1.0 and eps[-1] == 0.0
    assert np.all(T >= 0) and np.all(T <= 1 + 1e-12)
    assert np.all(np.diff(T) >= -1e-12)


def _isotropic(n, D, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, D))


@pytest.mark.parametrize("p_s", [0.1, 0.3])
def test_p9_isotropic_threshold_is_beta_quantile(p_s):
    """Isotropic Gaussian differences: f_d ~ Beta(d/2, (D-d)/2) for any orthonormal W."""
    D, M = 32, 40000
    X = _isotropic(2 * M, D, 5)
    mu, W, lam = pca.fit(_isotropic(4000, D, 7))   # W independent of the pairs
    pairs = np.stack([np.arange(0, 2 * M, 2), np.arange(1, 2 * M, 2)], 1)
    eps, T, _ = estimator.calibrate(X, W, lam, pairs, p_s)
    band = math.sqrt(math.log(2 / 1e-6) / (2 * M))  # DKW, failure prob 1e-6
    c = estimator.scale(lam)
    for d in (4, 8, 16, 24, 31):
        lo = stats.beta.ppf(1 - p_s - band, d / 2, (D - d) / 2)
        hi = stats.beta.ppf(1 - p_s + band, d / 2, (D - d) / 2)
        assert lo <= T[d - 1] <= hi, (d, lo, T[d - 1], hi)
        # literal form: 1 + eps_d = quantile of sqrt(c_d f_d)
        assert math.sqrt(c[d - 1] * lo) - 1 <= eps[d - 1] + 1e-12
        assert eps[d - 1] <= math.sqrt(c[d - 1] * hi) - 1 + 1e-12


def test_p10_low_rank_data_thresholds_are_one():
    rng = np.random.default_rng(9)
    D, rho = 20, 6
    X = rng.standard_normal((3000, rho)) @ rng.standard_normal((rho, D))
    mu, W, lam = pca.fit(X)
    pairs = workloads.calibration_pairs(len(X), 5000, seed=9)
    _, T, _ = estimator.calibrate(X, W, lam, pairs, 0.1)
    assert np.all(np.abs(T[rho - 1:] - 1.0) <= 1e-10)
    assert T[rho - 2] < 1.0


def test_p11_reduced_form_matches_literal_form():
    X, _ = workloads.make_mixture(4000, 32, 8, 1.2, 1, seed=4)
    mu, W, lam = pca.fit(X)
    pairs = workloads.calibration_pairs(len(X), 20000, seed=4)
    eps, T, _ = estimator.calibrate(X, W, lam, pairs, 0.1)
    np.testing.assert_allclose(estimator.thresholds_from_eps(eps, lam)[:-1], T[:-1], rtol=1e-12)
    rng = np.random.default_rng(0)
    c = estimator.scale(lam)
    S = rng.uniform(0, 50, (5000, 32))
    r = rng.uniform(1, 8, (5000, 1))
    lit = estimator.reject(estimator.estimate(S, c[None, :]), eps[None, :], r)
    red = S > T[None, :] * r ** 2
    margin = np.abs(c[None, :] * S - ((1 + eps[None, :]) * r) ** 2) / ((1 + eps[None, :]) * r) ** 2
    differ = (lit != red)[:, :-1]
    assert np.all(margin[:, :-1][differ] <= 1e-12)


def test_p16_exceedance_rate_on_fresh_pairs():
    X, _ = workloads.make_mixture(20000, 24, 16, 1.2, 1, seed=6)
    mu, W, lam = pca.fit(X)
    pairs = workloads.calibration_pairs(len(X), 20000, seed=6)
    _, T, _ = estimator.calibrate(X, W, lam, pairs, 0.2)
    fresh = workloads.calibration_pairs(len(X), 40000, seed=60)
    S, dis2 = estimator.pair_terms(X, W, fresh)
    rate = np.mean(S[:, :-1] > T[None, :-1] * dis2[:, None], axis=0)
    band = math.sqrt(math.log(2 / 1e-6) / (2 * 20000)) + math.sqrt(math.log(2 / 1e-6) / (2 * 40000))
    assert np.all(np.abs(rate - 0.2) <= band), rate


def test_duplicate_pairs_are_dropped():
    X = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 0.0], [0.0, 2.0]])
    mu, W, lam = pca.fit(X)
    pairs = np.array([[0, 1], [0, 2], [0, 3], [2, 3]])
    _, _, M = estimator.calibrate(X, W, lam, pairs, 0.1)
    assert M == 3
