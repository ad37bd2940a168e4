"""One distance comparison operation (DCO), in float64.

* Definition 1: given q, o and r, decide whether dis(q, o) <= r and if so return dis.
* Algorithm 1 (DADE): d starts at 0 and grows by Delta_d; at each step the estimate of
  Eq. (13) on the first d transformed dimensions is tested against (1 + eps_d) * r; a
  rejection before d = D ends the DCO with "no"; at d = D the estimate is the exact
  distance and is compared with r directly.
* FDScanning (Experiments, Algorithms): the exact full-D distance compared with r.

Reading where Algorithm 1 is silent: when Delta_d does not divide D the last step stops at
D (d <- min(d + Delta_d, D)), so tests happen only at d < D -- floor((D-1)/Delta_d) of them,
the count used by Lemma 5.
"""
from __future__ import annotations

import math

import numpy as np

from . import estimator


def dade_dco(o, q, r: float, delta_d: int, eps, c):
    """Algorithm 1 on transformed vectors o', q'.

    Returns (accepted, dis, d_exit): ``accepted`` is the DCO's answer, ``dis`` the exact
    distance when accepted (else None) and ``d_exit`` the number of dimensions used.
    ``eps[d-1]`` and ``c[d-1]`` are eps_d and c_d.
    """
    o = np.asarray(o, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    D = q.shape[0]
    d = 0
    while d < D:
        d = min(d + delta_d, D)
        S_d = float(np.sum((q[:d] - o[:d]) ** 2))
        dis_est = math.sqrt(c[d - 1] * S_d)
        if d < D:
            if bool(estimator.reject(dis_est, eps[d - 1], r)):
                return False, None, d
            continue
        # d == D: c_D = 1 and the estimate is the exact distance.
        return (dis_est <= r), (dis_est if dis_est <= r else None), d
    raise ValueError("empty vectors")


def fd_dco(o, q, r: float):
    """FDScanning: exact distance over all D dimensions, then compare with r."""
    dis = math.sqrt(float(np.sum((np.asarray(q, np.float64) - np.asarray(o, np.float64)) ** 2)))
    return (dis <= r), (dis if dis <= r else None), len(q)
