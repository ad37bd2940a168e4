"""Pins for the data-oblivious comparison (the random orthogonal projection of Figure 1): a
seeded Haar rotation in place of the data-aware W, with lambda_k the variance along each axis
and the same empirical calibration of eps_d."""
import numpy as np
import pytest

from oracle import ivf, pca
from paper_2411_17229_amd import workloads


@pytest.fixture(scope="module")
def data():
    X, _ = workloads.make_mixture(3000, 24, 8, 1.2, 1, seed=3)
    return X


def test_rotation_is_orthogonal_and_seeded():
    W = workloads.oblivious_rotation(32, seed=5)
    assert np.max(np.abs(W.T @ W - np.eye(32))) <= 1e-12
    np.testing.assert_array_equal(W, workloads.oblivious_rotation(32, seed=5))
    assert np.max(np.abs(W - workloads.oblivious_rotation(32, seed=6))) > 0.1


def test_axis_variances_are_the_eigenvalues_for_the_data_aware_w(data):
    # quadratic forms w_k^T E[YY^T] w_k against the eigendecomposition (Eq. (12))
    mu, W, lam = pca.fit(data)
    np.testing.assert_allclose(pca.axis_variances(data, mu, W), lam, rtol=1e-10, atol=1e-12)


def test_axis_variances_keep_the_trace(data):
    mu = pca.centre(data)
    v = pca.axis_variances(data, mu, workloads.oblivious_rotation(data.shape[1], seed=1))
    np.testing.assert_allclose(v.sum(), np.trace(pca.second_moment(data, mu)), rtol=1e-12)


def test_data_aware_prefix_variance_dominates(data):
    # Eq. (10) and the paragraph after it: for every d the data-aware W_d captures the most
    # variance of any orthonormal d-frame (Ky Fan), so its prefix sums bound the oblivious ones
    mu, _, lam = pca.fit(data)
    v = pca.axis_variances(data, mu, workloads.oblivious_rotation(data.shape[1], seed=2))
    assert np.all(np.cumsum(lam) >= np.cumsum(v) - 1e-9 * lam.sum())
    assert np.cumsum(lam)[3] > 1.2 * np.cumsum(v)[3]   # strictly, on this anisotropic mixture


def test_build_with_the_data_aware_w_is_the_default_build():
    w = workloads.WORKLOADS["small-20k-d128"]
    X, _ = workloads.make(w, n=4000)
    init = workloads.kmeans_init_rows(len(X), 16, w.seed)
    pairs = workloads.calibration_pairs(len(X), 5000, w.seed)
    a = ivf.build(X, 16, init, pairs, p_s=0.1, iters=3)
    b = ivf.build(X, 16, init, pairs, p_s=0.1, iters=3, rotation=a.W)
    np.testing.assert_allclose(b.lam, a.lam, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(b.T, a.T)   # the thresholds the test uses do not involve lambda
    np.testing.assert_allclose(b.eps, a.eps, rtol=1e-10)   # eps_d reads lambda (quadratic forms vs eigensolver)


def test_data_aware_test_reads_fewer_dimensions():
    # the paper's claim behind Figure 1 and the dimension-reduction study, on a small workload:
    # at the same P_s the data-aware transform rejects with fewer dimensions (tests every 8
    # dimensions, so that the dimensions read resolve the difference; 0.86 on this seed)
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n=6000, n_queries=12)
    init = workloads.kmeans_init_rows(len(X), 24, w.seed)
    pairs = workloads.calibration_pairs(len(X), 20000, w.seed)
    dims = {}
    for name, rot in (("pca", None), ("rop", workloads.oblivious_rotation(w.dim, w.seed))):
        oi = ivf.build(X, 24, init, pairs, p_s=0.1, iters=5, rotation=rot)
        _, _, logs = ivf.search(oi, Q, w.k, 6, 8, log=True)
        dims[name] = logs["dims"].sum() / logs["dcos"].sum()
    assert dims["pca"] < 0.9 * dims["rop"], dims
