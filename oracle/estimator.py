"""DADE estimate, calibrated deviation bound and hypothesis test, in float64.

Follows the Methodology section:
* Eq. (13): E||X1 - X2||^2 = (sum_{k<=D} lambda_k / sum_{k<=d} lambda_k) * E||W_d^T (X1 - X2)||^2.
  The estimate for one pair is dis'_d = sqrt(c_d * S_d) with c_d = Lambda_D / Lambda_d and
  S_d = ||W_d^T (x1 - x2)||^2 (reading: the scale multiplies the SQUARED distance, as in
  Eq. (13); Eq. (14) prints the scale inside the norm with garbled summation limits).
* Eq. (14): P{dis'/dis - 1 > eps_d} = P_s, with eps_d estimated from uniformly sampled data
  objects.  Reading: pairs of distinct data objects (passed in), pairs with dis = 0 dropped,
  eps_d + 1 = the ceil((1 - P_s) * M)-th smallest ratio dis'_d/dis (1-based, no interpolation).
* Hypothesis test: H0: dis < r is rejected iff dis' > (1 + eps_d) * r.

Reduced form (a reading, pinned against the literal one): because order statistics commute
with sqrt and with the positive constant c_d, rejecting is the same as S_d > T_d * r^2 where
T_d is the same order statistic of f_d = S_d / dis^2.  ``calibrate`` returns both eps_d (the
literal form, used by the oracle's tests) and T_d (the reduced form, imported by the GPU).
At d = D the test is never applied (Algorithm 1 compares exactly); T_D is set to 1 and
eps_D to 0, the values the exact identity c_D = 1, S_D = dis^2 gives.
"""
from __future__ import annotations

import math

import numpy as np


def prefix_variance(lam) -> np.ndarray:
    """Lambda_d = sum_{k<=d} lambda_k for d = 1..D (index d-1); Var(w_k^T X) = lambda_k by Eq. (12)."""
    return np.cumsum(np.asarray(lam, dtype=np.float64))


def scale(lam) -> np.ndarray:
    """c_d = Lambda_D / Lambda_d of Eq. (13) for d = 1..D (index d-1); c_D = 1."""
    L = prefix_variance(lam)
    c = L[-1] / L
    c[-1] = 1.0
    return c


def estimate(S_d, c_d):
    """dis'_d = sqrt(c_d * S_d) (Eq. (13), one pair)."""
    return np.sqrt(np.asarray(c_d, dtype=np.float64) * np.asarray(S_d, dtype=np.float64))


def reject(dis_est, eps_d, r):
    """True iff H0 (dis < r) is rejected: dis' > (1 + eps_d) * r.  r may be +inf."""
    with np.errstate(invalid="ignore"):
        return np.asarray(dis_est) > (1.0 + np.asarray(eps_d)) * r


def order_statistic_index(p: float, m: int) -> int:
    """1-based index ceil(p * m), clamped to [1, m]."""
    return min(max(int(math.ceil(p * m)), 1), m)


def order_statistic(values, p: float, axis=0):
    """The ceil(p*M)-th smallest entry along ``axis`` (1-based, no interpolation)."""
    v = np.sort(np.asarray(values, dtype=np.float64), axis=axis)
    k = order_statistic_index(p, v.shape[axis])
    return np.take(v, k - 1, axis=axis)


def pair_terms(X, W, pairs, stored=None):
    """(S, dis2) for calibration pairs.

    S[i, d-1] = ||W_d^T (x_a - x_b)||^2 and dis2[i] = ||x_a - x_b||^2, both in float64 from the
    original vectors.  With ``stored`` (rotated coordinates as held by a low-precision index),
    S is taken from stored[a] - stored[b] instead while dis2 stays exact.
    Pairs with dis2 == 0 are dropped.
    """
    X = np.asarray(X)
    a, b = np.asarray(pairs)[:, 0], np.asarray(pairs)[:, 1]
    dx = X[a].astype(np.float64) - X[b].astype(np.float64)
    dis2 = np.einsum("ij,ij->i", dx, dx)
    keep = dis2 > 0
    if stored is None:
        y = dx[keep] @ np.asarray(W, dtype=np.float64)
    else:
        st = np.asarray(stored)
        y = st[a[keep]].astype(np.float64) - st[b[keep]].astype(np.float64)
    return np.cumsum(y * y, axis=1), dis2[keep]


def calibrate(X, W, lam, pairs, p_s: float, stored=None):
    """eps_d (Eq. (14), literal form) and T_d (reduced form) for d = 1..D.

    Returns (eps, T, M) with M the number of pairs used.
    """
    S, dis2 = pair_terms(X, W, pairs, stored)
    M = S.shape[0]
    c = scale(lam)
    ratio = estimate(S, c[None, :]) / np.sqrt(dis2)[:, None]
    eps = order_statistic(ratio, 1.0 - p_s, axis=0) - 1.0
    T = order_statistic(S / dis2[:, None], 1.0 - p_s, axis=0)
    eps[-1] = 0.0
    T[-1] = 1.0
    return eps, T, M


def thresholds_from_eps(eps, lam) -> np.ndarray:
    """T_d = (1 + eps_d)^2 / c_d: the reduced-form multiplier equivalent to eps_d."""
    return (1.0 + np.asarray(eps, dtype=np.float64)) ** 2 / scale(lam)
