"""Brute-force K nearest neighbours in float64 (ground truth; Problem setting of the Introduction).

Results are ordered by (squared distance, id).  Small problems use explicit differences
(the definition); larger ones use the expansion ||x||^2 - 2 x.q + ||q||^2 in float64 with
chunking, whose rounding (~1e-15 relative) is far below any tolerance used with it.
"""
from __future__ import annotations

import numpy as np


def _topk_rows(d2, ids, k):
    out_i = np.full((d2.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((d2.shape[0], k), np.inf)
    for r in range(d2.shape[0]):
        o = np.lexsort((ids, d2[r]))[:k]
        out_i[r, :len(o)] = ids[o]
        out_d[r, :len(o)] = d2[r, o]
    return out_i, out_d


def brute_force(X, Q, k: int, direct_limit: int = 200_000_000, chunk: int = 65_536):
    """(ids [nq, k], dist2 [nq, k]) of the exact K nearest rows of X for every query."""
    X = np.asarray(X)
    Q = np.asarray(Q, dtype=np.float64)
    n = X.shape[0]
    if n * X.shape[1] * Q.shape[0] <= direct_limit:
        Xd = X.astype(np.float64)
        d2 = np.stack([np.sum((Xd - q) ** 2, axis=1) for q in Q])
        return _topk_rows(d2, np.arange(n, dtype=np.int64), k)
    best_i = np.full((Q.shape[0], 0), -1, dtype=np.int64)
    best_d = np.full((Q.shape[0], 0), np.inf)
    qn = np.einsum("ij,ij->i", Q, Q)
    for s in range(0, n, chunk):
        Xc = X[s:s + chunk].astype(np.float64)
        xn = np.einsum("ij,ij->i", Xc, Xc)
        d2 = np.maximum(qn[:, None] - 2.0 * (Q @ Xc.T) + xn[None, :], 0.0)
        kk = min(k, d2.shape[1])
        part = np.argpartition(d2, kk - 1, axis=1)[:, :kk] if d2.shape[1] > kk else \
            np.tile(np.arange(d2.shape[1]), (Q.shape[0], 1))
        cand_d = np.concatenate([best_d, np.take_along_axis(d2, part, 1)], axis=1)
        cand_i = np.concatenate([best_i, part + s], axis=1)
        new_i = np.empty((Q.shape[0], min(k, cand_d.shape[1])), dtype=np.int64)
        new_d = np.empty_like(new_i, dtype=np.float64)
        for r in range(Q.shape[0]):
            o = np.lexsort((cand_i[r], cand_d[r]))[:new_i.shape[1]]
            new_i[r] = cand_i[r, o]
            new_d[r] = cand_d[r, o]
        best_i, best_d = new_i, new_d
    out_i = np.full((Q.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((Q.shape[0], k), np.inf)
    out_i[:, :best_i.shape[1]] = best_i
    out_d[:, :best_d.shape[1]] = best_d
    return out_i, out_d


def recall(found_ids, gt_ids, k: int) -> np.ndarray:
    """|result ∩ GT| / K per query (Experiments, Performance Metrics)."""
    out = np.empty(len(gt_ids))
    for i, (f, g) in enumerate(zip(found_ids, gt_ids)):
        out[i] = len(set(int(x) for x in f[:k] if x >= 0) & set(int(x) for x in g[:k])) / k
    return out
