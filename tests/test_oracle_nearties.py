"""Pins for the oracle's rerank rules, its rerank margin, the probe order's tie rule and the
near-tie protocol (decisions logged within a margin, re-runs with a decision taken the other
way), each against a hand-worked case or a property that fixes it."""
import math

import numpy as np
import pytest

from oracle import estimator, ivf, lowp
from paper_2411_17229_amd import workloads


def test_rerank_margin_is_the_order_statistic_of_relative_errors():
    """Pairs built so that pair i has ||x_a - x_b||^2 = 1 and stored-precision S_D = 1 + e_i:
    the relative errors are the e_i, so delta is the ceil(p M)-th smallest e_i (1-based)."""
    rng = np.random.default_rng(4)
    M = 1000
    e = rng.permutation(np.arange(1, M + 1) / M)          # relative errors 0.001 .. 1.0
    e[::7] *= -1.0                                          # some stored distances below the exact
    X = np.zeros((2 * M, 2))
    X[1::2, 0] = 1.0                                        # each pair one unit apart
    st = np.zeros((2 * M, 2))
    st[1::2, 0] = np.sqrt(1.0 + e)                          # stored difference: S_D = 1 + e_i
    pairs = np.stack([np.arange(0, 2 * M, 2), np.arange(1, 2 * M, 2)], 1)
    srt = np.sort(np.abs(e))
    assert abs(lowp.rerank_margin(X, pairs, st) - srt[math.ceil(0.999 * M) - 1]) < 1e-12
    assert abs(lowp.rerank_margin(X, pairs, st, quantile=0.5) - srt[499]) < 1e-12
    assert abs(lowp.rerank_margin(X, pairs, st, quantile=1.0) - 1.0) < 1e-12
    # a pair of equal vectors is dropped, not counted as an error
    X2, st2 = np.vstack([X, [[5.0, 5.0], [5.0, 5.0]]]), np.vstack([st, [[9.0, 9.0], [0.0, 0.0]]])
    pairs2 = np.vstack([pairs, [[2 * M, 2 * M + 1]]])
    assert abs(lowp.rerank_margin(X2, pairs2, st2) - srt[math.ceil(0.999 * M) - 1]) < 1e-12


def test_probe_order_breaks_distance_ties_by_list_id():
    """Integer centroids at exactly equal distances from q: order by list id among ties; the
    order is the sort of (dist^2, id) pairs written out by hand."""
    cent = np.array([[0, 2], [1, 0], [-1, 0], [3, 0], [0, -1], [0, 1], [2, 0], [-2, 0]], dtype=np.float64)
    q = np.zeros(2)
    order, d2 = ivf.probe_order(q, cent, 8)
    assert list(order) == [1, 2, 4, 5, 0, 6, 7, 3]      # distances 1,1,1,1 then 4,4,4 then 9
    assert list(d2) == [1, 1, 1, 1, 4, 4, 4, 9]
    assert list(ivf.probe_order(q, cent, 3)[0]) == [1, 2, 4]
    # relabelling the lists permutes the ids but keeps the rule
    perm = np.array([3, 7, 0, 5, 1, 6, 2, 4])
    order2, _ = ivf.probe_order(q, cent[np.argsort(perm)], 8)
    assert list(order2[:4]) == sorted(perm[[1, 2, 4, 5]])


def _index_2d(rows, offsets, cent, lam=(1.0, 1.0), eps=(0.0, 0.0)):
    rows = np.asarray(rows, float)
    return ivf.Index(np.zeros(2), np.eye(2), np.array(lam), np.array(eps), np.asarray(cent, float),
                     np.asarray(offsets), np.arange(len(rows)), rows)


def test_cut_tie_is_logged_and_flipped():
    """K = 1 over rows at squared distances 1 and 1 + 1e-9: the cut between them is a near tie
    (gap 1e-9); the re-run with the cut flipped returns the second row."""
    idx = _index_2d([[1.0, 0.0], [0.0, math.sqrt(1 + 1e-9)]], [0, 2], [[0.0, 0.0]])
    q = np.zeros((1, 2))
    ids, _, logs = ivf.search(idx, q, 1, 1, 1, mode="exact", log=True, event_tol=1e-6)
    assert ids[0, 0] == 0
    ev = logs["events"][0]
    cut = [k for m, k in ev if k[0] == "cut"]
    assert cut == [("cut", 0, 0, 1)] and abs(ev[0][0] - 1e-9) < 1e-12
    ids2, d2 = ivf.search(idx, q, 1, 1, 1, mode="exact", flips={0: {cut[0]}})
    assert ids2[0, 0] == 1 and abs(d2[0, 0] - (1 + 1e-9)) < 1e-15
    # a tie farther than event_tol is not logged
    _, _, logs = ivf.search(idx, q, 1, 1, 1, mode="exact", log=True, event_tol=1e-10)
    assert not [k for m, k in logs["events"][0] if k[0] == "cut"]


def test_keep_compare_is_logged_and_flipped():
    """K = 1, fill_min 0: round 0 holds row 0 (d^2 = 1); row 1 (d^2 = 1 - 1e-8) is kept by the
    keep compare of round 1 with margin 1e-8; flipped, it is not kept."""
    idx = _index_2d([[1.0, 0.0], [math.sqrt(1 - 1e-8), 0.0]], [0, 1, 2], [[0.1, 0.0], [0.2, 0.0]])
    q = np.zeros((1, 2))
    kw = dict(mode="exact", fill_min=0, growth=0)
    ids, _, logs = ivf.search(idx, q, 1, 2, 1, log=True, event_tol=1e-6, **kw)
    assert ids[0, 0] == 1
    keys = [k for m, k in logs["events"][0]]
    assert ("keep", 1, 1) in keys
    ids2, _ = ivf.search(idx, q, 1, 2, 1, flips={0: {("keep", 1, 1)}}, **kw)
    assert ids2[0, 0] == 0


def test_test_decision_is_logged_and_flipped():
    """D = 2, Delta_d = 1, T_1 = 0.5 (eps_1 from it with lambda = (1, 1)): the heap holds d^2 = 1
    (r^2 = 1); row 1 = (sqrt(0.5 + 1e-9), 0.5) has S_1 = 0.5 + 1e-9 > T_1 r^2 = 0.5 and is
    rejected at d = 1 with margin about 2e-9; flipped, it is tested in full and kept (d^2 =
    0.75 + 1e-9 < 1)."""
    lam = np.array([1.0, 1.0])
    T1 = 0.5
    eps = np.array([math.sqrt(T1 * estimator.scale(lam)[0]) - 1.0, 0.0])
    idx = _index_2d([[1.0, 0.0], [math.sqrt(0.5 + 1e-9), 0.5]], [0, 1, 2], [[0.1, 0.0], [0.2, 0.0]], lam, eps)
    q = np.zeros((1, 2))
    kw = dict(fill_min=0, growth=0)
    ids, _, logs = ivf.search(idx, q, 1, 2, 1, log=True, event_tol=1e-6, **kw)
    assert ids[0, 0] == 0 and logs["dims"][0] == 2 + 1
    keys = [k for m, k in logs["events"][0]]
    assert ("test", 1, 1, 1) in keys
    ids2, d2, logs2 = ivf.search(idx, q, 1, 2, 1, log=True, flips={0: {("test", 1, 1, 1)}}, **kw)
    assert ids2[0, 0] == 1 and logs2["dims"][0] == 2 + 2
    assert abs(d2[0, 0] - (0.75 + 1e-9)) < 1e-15


def test_probe_gap_is_logged_and_flipped():
    """Two lists whose centroids lie at squared distances 1 and 1 + 1e-9 from q; nprobe 1 scans
    the nearer one; the flipped probe order scans the other."""
    idx = _index_2d([[1.0, 0.0], [0.0, 3.0]], [0, 1, 2], [[1.0, 0.0], [0.0, math.sqrt(1 + 1e-9)]])
    q = np.zeros((1, 2))
    ids, _, logs = ivf.search(idx, q, 1, 1, 1, mode="exact", log=True, event_tol=1e-6)
    assert ids[0, 0] == 0 and ("probe", 0) in [k for m, k in logs["events"][0]]
    assert logs["probe_gap"][0] < 1e-8
    ids2, _ = ivf.search(idx, q, 1, 1, 1, mode="exact", flips={0: {("probe", 0)}})
    assert ids2[0, 0] == 1


def test_gate_and_lazy_bound_are_logged_and_flipped():
    """The hand-worked lazy case where the bound skips id 4 (stored 1.134225 against
    (1 + 0.1) x 1.0201 = 1.12211): the skip is a logged 'bound' decision; flipped, id 4 is
    reranked and the lazy rule returns what the plain rule returns."""
    Ys = np.array([[1, 0], [1.1, 0], [0, 1.03], [0, 1.04], [0, 1.065]], float)
    Ye = np.array([[1, 0], [1.1, 0], [1.01, 0], [1.02, 0], [1.005, 0]], float)
    idx = ivf.Index(np.zeros(2), np.eye(2), np.array([1.0, 1.0]), np.zeros(2),
                    np.array([[0.1, 0.0], [5.0, 5.0]]), np.array([0, 2, 5]), np.arange(5), Ys,
                    Y_exact=Ye, delta=0.1)
    q = np.zeros((1, 2))
    kw = dict(mode="exact", fill_min=0, growth=0, rerank="lazy")
    ids, _, logs = ivf.search(idx, q, 2, 2, 1, log=True, event_tol=0.05, **kw)
    assert list(ids[0]) == [0, 2]
    keys = [k for m, k in logs["events"][0]]
    assert ("bound", 1, 4) in keys and ("gate", 1, 4) not in keys   # gate 1.331: margin 0.148
    ids2, _ = ivf.search(idx, q, 2, 2, 1, flips={0: {("bound", 1, 4)}}, **kw)
    assert list(ids2[0]) == [0, 4]
    ids3, _ = ivf.search(idx, q, 2, 2, 1, mode="exact", fill_min=0, growth=0, rerank="all")
    assert list(ids3[0]) == [0, 4]
    # the gate: flipped for id 4, it is dropped before any rerank
    ids4, _ = ivf.search(idx, q, 2, 2, 1, mode="exact", fill_min=0, growth=0, rerank="all",
                         flips={0: {("gate", 1, 4)}})
    assert list(ids4[0]) == [0, 2]


@pytest.mark.slow
def test_lazy_rule_equals_plain_rule_without_delta_tail():
    """A skewed high-D mixture with a BF16 store (the bench's setting, smaller): the lazy rule
    returns exactly what the plain rule returns for every query none of whose probed candidates
    has a stored-precision error of S_D above delta (the rule's correctness condition); over
    all queries the two differ rarely."""
    X, Q = workloads.make_mixture(8000, 192, 64, 1.5, 80, seed=31)
    init = workloads.kmeans_init_rows(len(X), 32, 31)
    pairs = workloads.calibration_pairs(len(X), 40000, 31)
    idx = ivf.build(X, 32, init, pairs, p_s=0.01, store=lambda y: lowp.store(y, "bf16"))
    kw = dict(schedule="doubling", fill_min=32, growth=0)
    a_i, a_d = ivf.search(idx, Q, 10, 6, 32, rerank="all", **kw)
    b_i, b_d = ivf.search(idx, Q, 10, 6, 32, rerank="lazy", **kw)
    cent = idx.cent_rot()
    Qr = (Q - idx.mu) @ idx.W
    tail_queries = differ = 0
    for qi in range(len(Q)):
        probes, _ = ivf.probe_order(Qr[qi], cent, 6)
        cand = np.concatenate([idx.ids[idx.offsets[l]:idx.offsets[l + 1]] for l in probes])
        SD = np.sum((idx.Y[cand] - Qr[qi]) ** 2, axis=1)
        ex = np.sum((idx.Y_exact[cand] - Qr[qi]) ** 2, axis=1)
        tail = np.any(np.abs(SD - ex) / ex > idx.delta)
        tail_queries += int(tail)
        same = np.array_equal(a_i[qi], b_i[qi])
        differ += int(not same)
        if not tail:
            assert same, qi
            np.testing.assert_array_equal(a_d[qi], b_d[qi])
    assert differ <= tail_queries and differ <= 0.05 * len(Q), (differ, tail_queries)
