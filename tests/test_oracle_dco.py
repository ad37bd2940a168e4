"""Pins for oracle.dco: hand-worked Algorithm 1 cases and Lemma 5's failure bound."""
import math
import os

import numpy as np
import pytest

from oracle import dco, estimator, pca
from paper_2411_17229_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dco_cases.txt")
LAM = np.array([4.0, 3.0, 2.0, 1.0])
EPS = np.array([0.5, 0.1, 0.05, 0.0])


def _cases():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, dd, r, o, acc, dis, dexit = [f.strip() for f in line.split("|")]
        yield pytest.param(int(dd), float(r), np.array(o.split(), float), acc == "1",
                           None if dis == "-" else float(dis), int(dexit), id=name)


@pytest.mark.parametrize("dd,r,o,acc,dis,dexit", list(_cases()))
def test_hand_worked_algorithm1(dd, r, o, acc, dis, dexit):
    ok, got_dis, got_d = dco.dade_dco(o, np.zeros(4), r, dd, EPS, estimator.scale(LAM))
    assert ok == acc
    assert got_d == dexit
    if dis is None:
        assert got_dis is None
    else:
        assert abs(got_dis - dis) <= 1e-12 * dis


def test_fdscanning_by_hand():
    assert dco.fd_dco([3, 4], [0, 0], 5.0) == (True, 5.0, 2)
    assert dco.fd_dco([3, 4], [0, 0], 4.99)[0] is False


@pytest.fixture(scope="module")
def calibrated():
    X, _ = workloads.make_mixture(6000, 32, 8, 1.2, 1, seed=11)
    mu, W, lam = pca.fit(X)
    pairs = workloads.calibration_pairs(len(X), 20000, seed=11)
    eps, T, _ = estimator.calibrate(X, W, lam, pairs, 0.1)
    return X, mu, W, lam, eps


def test_lemma5_no_failure_when_dis_above_r(calibrated):
    """dis > r: Algorithm 1 never answers yes (a rejection is always correct)."""
    X, mu, W, lam, eps = calibrated
    Y = pca.rotate(X, mu, W)
    c = estimator.scale(lam)
    rng = np.random.default_rng(1)
    for _ in range(400):
        i, j = rng.integers(0, len(X), 2)
        dis = math.sqrt(np.sum((Y[i] - Y[j]) ** 2))
        if dis == 0:
            continue
        r = dis * rng.uniform(0.5, 0.999)
        for dd in (1, 4, 8, 32):
            assert dco.dade_dco(Y[i], Y[j], r, dd, eps, c)[0] is False


@pytest.mark.parametrize("dd", [4, 8])
def test_lemma5_failure_bound_when_dis_at_most_r(calibrated, dd):
    """dis <= r: failure rate <= floor((D-1)/Delta_d) * P_s on held-out pairs (r = dis)."""
    X, mu, W, lam, eps = calibrated
    Y = pca.rotate(X, mu, W)
    c = estimator.scale(lam)
    fresh = workloads.calibration_pairs(len(X), 3000, seed=12)
    fails = 0
    for i, j in fresh:
        dis = math.sqrt(np.sum((Y[i] - Y[j]) ** 2))
        ok, got, _ = dco.dade_dco(Y[i], Y[j], dis * (1 + 1e-12), dd, eps, c)
        fails += not ok
        if ok:
            assert abs(got - dis) <= 1e-12 * dis
    bound = ((32 - 1) // dd) * 0.1
    rate = fails / len(fresh)
    assert rate <= bound
    # each test alone fails with probability about P_s, so at least one test's worth shows up
    assert rate >= 0.1 - 3 * math.sqrt(0.1 * 0.9 / len(fresh))


def test_rejection_is_strict():
    """lambda = (1,1,1,1): c_2 = 2; eps_2 = 0; o' = (1,1,0,0), q' = 0: at d = 2, S = 2 and
    dis' = sqrt(2*2) = 2 = (1 + 0) * r for r = 2, so H0 is NOT rejected (the event is
    dis' > (1+eps) r); at d = 4, dis = sqrt(2) <= 2 -> yes.  With r just below 2 it is rejected."""
    c = estimator.scale([1.0, 1.0, 1.0, 1.0])
    eps = np.zeros(4)
    ok, dis, d = dco.dade_dco([1, 1, 0, 0], np.zeros(4), 2.0, 2, eps, c)
    assert ok and d == 4 and abs(dis - math.sqrt(2)) < 1e-15
    ok, dis, d = dco.dade_dco([1, 1, 0, 0], np.zeros(4), np.nextafter(2.0, 0), 2, eps, c)
    assert not ok and d == 2
