"""Property tests of the IVF oracle (hypothesis) on tiny random inputs with the edge cases the
method has: duplicate rows, exact distance ties (small integer coordinates), K larger than the
candidate count, lists left empty by k-means, and D not a multiple of Delta_d.

* FDScanning over every list is brute-force KNN (oracle/knn.py): the same distances, and the
  same ids wherever a distance is not tied with its neighbour in the order.
* Every DADE result is well formed: valid distinct ids, (-1, +inf) padding only at the end,
  exactly min(K, n) results when every list is probed, rows ascending, distances exact.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import ivf, knn

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def make_case(n, d, nlist, seed, dup):
    rng = np.random.default_rng(seed)
    X = rng.integers(-3, 4, (n, d)).astype(np.float32)
    if dup:
        X[n // 2] = X[0]
    if len(np.unique(X, axis=0)) < 2:
        X[1] = X[0] + 1.0
    nlist = min(nlist, n)
    init = rng.choice(n, nlist, replace=False)
    a, b = rng.integers(0, n, 400), rng.integers(0, n, 400)
    pairs = np.stack([a, b], 1)[a != b]
    keep = np.any(X[pairs[:, 0]] != X[pairs[:, 1]], axis=1)
    if not keep.any():   # calibration needs one pair of distinct rows
        i, j = np.nonzero(np.any(X[:, None] != X[None, :], axis=2))
        pairs = np.array([[i[0], j[0]]])
    oi = ivf.build(X, nlist, init, pairs, p_s=0.1, iters=3)
    Q = rng.integers(-3, 4, (4, d)).astype(np.float32)
    return X, Q, oi


CASES = dict(n=st.integers(2, 40), d=st.integers(1, 12), nlist=st.integers(1, 6), K=st.integers(1, 50),
             dd=st.integers(1, 12), dup=st.booleans(), seed=st.integers(0, 10 ** 6))
SETTINGS = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(**CASES)
def test_exact_mode_over_all_lists_is_brute_force(n, d, nlist, K, dd, dup, seed):
    X, Q, oi = make_case(n, d, nlist, seed, dup)
    ids, d2 = ivf.search(oi, Q, K, oi.nlist, min(dd, d), mode="full_d", schedule="doubling")
    bi, bd = knn.brute_force(X, Q, K + 1)   # one more: a tie across the K-th place counts too
    np.testing.assert_allclose(d2, bd[:, :K], rtol=1e-9, atol=1e-9)
    for q in range(len(Q)):
        for j in range(min(K, n)):
            tied = any(abs(bd[q, j] - bd[q, i]) <= 1e-9 for i in (j - 1, j + 1) if 0 <= i < min(K + 1, n))
            if not tied:
                assert ids[q, j] == bi[q, j], (q, j)


@SETTINGS
@given(schedule=st.sampled_from(["per_rank", "doubling", "sequential"]), **CASES)
def test_dade_results_are_well_formed(n, d, nlist, K, dd, dup, seed, schedule):
    X, Q, oi = make_case(n, d, nlist, seed, dup)
    ids, d2 = ivf.search(oi, Q, K, oi.nlist, min(dd, d), mode="dade", schedule=schedule)
    Xd = X.astype(np.float64)
    for q in range(len(Q)):
        valid = ids[q] >= 0
        m = int(valid.sum())
        assert m <= min(K, n)
        assert np.all(valid[:m]) and not np.any(valid[m:]) and np.all(np.isinf(d2[q, m:]))
        assert len(set(ids[q, :m].tolist())) == m
        ex = np.sum((Xd[ids[q, :m]] - Q[q].astype(np.float64)) ** 2, axis=1)
        np.testing.assert_allclose(d2[q, :m], ex, rtol=1e-9, atol=1e-9)
        assert np.all(np.diff(d2[q, :m]) >= -1e-9)
        # the heap fills before any test can reject: at least min(K, n) candidates are scanned
        # whenever every list is probed, so the first round alone keeps min(K, n) of them
        assert m == min(K, n)
