"""Pins for oracle.pca (Lemma 1, Lemma 2, Eqs. (10)-(12)) against closed forms and SVD."""
import os

import numpy as np
import pytest

from oracle import pca
from paper_2411_17229_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pca_cases.txt")


def _golden():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        _, pts, mean, lam, W = [f.strip() for f in line.split("|")]
        P = np.array([[float(v) for v in p.split()] for p in pts.split(";")])
        Wc = np.array([[float(v) for v in p.split()] for p in W.split(";")]).T
        yield P, np.array(mean.split(), float), np.array(lam.split(), float), Wc


@pytest.fixture(scope="module")
def data():
    X, _ = workloads.make_mixture(3000, 24, 8, 1.2, 1, seed=3)
    return X


@pytest.mark.parametrize("case", list(_golden()))
def test_closed_form_cases(case):
    P, mean, lam, W = case
    mu, Wo, lo = pca.fit(P)
    np.testing.assert_allclose(mu, mean, atol=1e-12)
    np.testing.assert_allclose(lo, lam, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Wo, W, atol=1e-12)


def test_p1_orthonormal(data):
    _, W, _ = pca.fit(data)
    assert np.max(np.abs(W.T @ W - np.eye(W.shape[0]))) <= 1e-12


def test_p2_rotation_preserves_distances(data):
    mu, W, _ = pca.fit(data)
    Y = pca.rotate(data, mu, W)
    rng = np.random.default_rng(0)
    a, b = rng.integers(0, len(data), 500), rng.integers(0, len(data), 500)
    d_orig = np.sum((data[a].astype(np.float64) - data[b]) ** 2, axis=1)
    d_rot = np.sum((Y[a] - Y[b]) ** 2, axis=1)
    m = d_orig > 0
    assert np.max(np.abs(d_rot[m] - d_orig[m]) / d_orig[m]) <= 1e-12


def test_p3_lemma2_variance_sum(data):
    _, _, lam = pca.fit(data)
    total = np.sum(np.var(data.astype(np.float64), axis=0))
    assert abs(lam.sum() - total) / total <= 1e-12


def test_p4_eq12_rotated_covariance_is_diag_lambda(data):
    mu, W, lam = pca.fit(data)
    Y = pca.rotate(data, mu, W)
    Cy = (Y - Y.mean(0)).T @ (Y - Y.mean(0)) / len(Y)
    np.testing.assert_allclose(np.diag(Cy), lam, rtol=1e-10)
    off = Cy - np.diag(np.diag(Cy))
    assert np.max(np.abs(off)) <= 1e-12 * lam[0]
    assert np.all(np.diff(lam) <= 0)          # Eq. (11): k-th LARGEST eigenvalue first


def test_p5_pca_equals_svd_of_centred_data(data):
    X = data.astype(np.float64)
    Xc = X - X.mean(0)
    _, s, Vt = np.linalg.svd(Xc, full_matrices=False)
    _, W, lam = pca.fit(data)
    np.testing.assert_allclose(lam, s ** 2 / len(X), rtol=1e-10)
    gap = np.abs(np.diff(s ** 2)) / (s[:-1] ** 2)
    for k in range(len(s) - 1):
        if gap[k] > 1e-3 and (k == 0 or gap[k - 1] > 1e-3):
            assert abs(abs(W[:, k] @ Vt[k]) - 1.0) < 1e-8


def test_lemma1_shift_invariance(data):
    mu, W, lam = pca.fit(data)
    mu2, W2, lam2 = pca.fit(data.astype(np.float64) + 123.0)
    np.testing.assert_allclose(lam2, lam, rtol=1e-8)
    np.testing.assert_allclose(mu2, mu + 123.0, rtol=1e-12)


def test_sign_rule():
    V = np.array([[0.6, -0.8], [-0.8, -0.6]])
    F = pca.fix_signs(V)
    assert F[1, 0] > 0 and F[0, 1] > 0
