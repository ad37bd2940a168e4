"""Pins for oracle.ivf and oracle.knn: k-means against scikit-learn, brute force against
scipy, exact IVF against brute force, schedule invariance, the scalar transcription of
Algorithm 1 + heap against the vectorised search, and the result invariants."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import ivf, knn, lowp
from paper_2411_17229_amd import workloads

N, D, NLIST = 3000, 32, 16


@pytest.fixture(scope="module")
def setup():
    X, Q = workloads.make_mixture(N, D, 12, 1.2, 12, seed=21)
    init = workloads.kmeans_init_rows(N, NLIST, seed=21)
    pairs = workloads.calibration_pairs(N, 20000, seed=21)
    index = ivf.build(X, NLIST, init, pairs, p_s=0.1, iters=10)
    return X, Q, init, index


def test_kmeans_matches_sklearn_lloyd(setup):
    from sklearn.cluster import KMeans
    X, _, init, index = setup
    km = KMeans(n_clusters=NLIST, init=X[init].astype(np.float64), n_init=1, max_iter=10,
                tol=0.0, algorithm="lloyd").fit(X.astype(np.float64))
    np.testing.assert_allclose(index.centroids, km.cluster_centers_, rtol=1e-9, atol=1e-9)


def test_assign_is_nearest_centroid(setup):
    X, _, _, index = setup
    lab = ivf.assign(X, index.centroids)
    ref = np.argmin(cdist(X.astype(np.float64), index.centroids, "sqeuclidean"), axis=1)
    assert np.array_equal(lab, ref)


def test_lists_partition_rows_in_ascending_order(setup):
    X, _, _, index = setup
    assert index.offsets[0] == 0 and index.offsets[-1] == N
    assert np.array_equal(np.sort(index.ids), np.arange(N))
    lab = ivf.assign(X, index.centroids)
    for l in range(NLIST):
        seg = index.ids[index.offsets[l]:index.offsets[l + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(lab[seg] == l)


def test_brute_force_matches_scipy():
    X, Q = workloads.make_mixture(500, 8, 4, 1.0, 5, seed=3)
    ids, d2 = knn.brute_force(X, Q, 7)
    ref = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    for i in range(len(Q)):
        o = np.lexsort((np.arange(500), ref[i]))[:7]
        assert np.array_equal(ids[i], o)
        np.testing.assert_allclose(d2[i], ref[i, o], rtol=1e-12)
    # the chunked expansion path agrees with the direct one
    ids2, d22 = knn.brute_force(X, Q, 7, direct_limit=0, chunk=128)
    assert np.array_equal(ids2, ids)
    np.testing.assert_allclose(d22, d2, rtol=1e-10)


def test_p12_exact_ivf_all_lists_is_brute_force(setup):
    X, Q, _, index = setup
    for K in (1, 10, 25):
        ids, d2 = ivf.search(index, Q, K, NLIST, 8, mode="exact")
        gi, gd = knn.brute_force(X, Q, K)
        assert np.array_equal(ids, gi)
        np.testing.assert_allclose(d2, gd, rtol=1e-10)


def test_p13_exact_mode_is_schedule_invariant(setup):
    X, Q, _, index = setup
    res = [ivf.search(index, Q, 10, 5, 8, mode="exact", schedule=s)
           for s in ("per_rank", "doubling", "sequential")]
    for ids, d2 in res[1:]:
        assert np.array_equal(ids, res[0][0])
    # one global round over the probed candidates = the 10 nearest of those candidates
    for qi in range(len(Q)):
        probes, _ = ivf.probe_order((Q[qi] - index.mu) @ index.W, index.cent_rot(), 5)
        cand = np.concatenate([index.ids[index.offsets[l]:index.offsets[l + 1]] for l in probes])
        d = np.sum((X[cand].astype(np.float64) - Q[qi]) ** 2, axis=1)
        o = np.lexsort((cand, d))[:10]
        assert np.array_equal(res[0][0][qi], cand[o])


@pytest.mark.parametrize("mode,dd", [("dade", 8), ("dade", 5), ("exact", 8)])
def test_p14_scalar_algorithm1_heap_matches_vectorised_sequential(setup, mode, dd):
    X, Q, _, index = setup
    a_i, a_d, a_log = ivf.search_scalar(index, Q[:6], 10, 3, dd, mode=mode, log=True)
    b_i, b_d, b_log = ivf.search(index, Q[:6], 10, 3, dd, mode=mode, schedule="sequential", log=True)
    assert np.array_equal(a_i, b_i)
    np.testing.assert_allclose(a_d, b_d, rtol=1e-12)
    # every DCO exits at the same d and the same candidates are kept
    assert np.array_equal(a_log["dims"], b_log["dims"])
    assert np.array_equal(a_log["accepted"], b_log["accepted"])
    if mode == "dade":
        assert a_log["dims"].sum() < b_log["dcos"].sum() * D


@pytest.mark.parametrize("schedule", ["per_rank", "doubling", "sequential"])
def test_result_invariants(setup, schedule):
    """I1 exact distances, I2 DADE >= exact IVF elementwise, I3 recall <= exact IVF, I4 counts."""
    X, Q, _, index = setup
    K, npb = 10, 4
    ids, d2, logs = ivf.search(index, Q, K, npb, 8, schedule=schedule, log=True)
    ei, ed = ivf.search(index, Q, K, npb, 8, mode="exact")
    gi, _ = knn.brute_force(X, Q, K)
    for qi in range(len(Q)):
        v = ids[qi] >= 0
        exact = np.sum((X[ids[qi][v]].astype(np.float64) - Q[qi]) ** 2, axis=1)
        np.testing.assert_allclose(d2[qi][v], exact, rtol=1e-12)
        assert np.all(np.sort(d2[qi]) >= np.sort(ed[qi]) - 1e-12 * np.abs(ed[qi]))
    assert np.all(knn.recall(ids, gi, K) <= knn.recall(ei, gi, K) + 1e-12)
    cent = index.cent_rot()
    for qi in range(len(Q)):
        probes, _ = ivf.probe_order((Q[qi] - index.mu) @ index.W, cent, npb)
        n_cand = sum(index.offsets[l + 1] - index.offsets[l] for l in probes)
        assert logs["dcos"][qi] == n_cand
        assert logs["dims"][qi] <= n_cand * D


def test_dade_reads_fewer_dims_and_keeps_recall(setup):
    X, Q, _, index = setup
    ids, _, logs = ivf.search(index, Q, 10, 8, 4, log=True)
    gi, _ = knn.brute_force(X, Q, 10)
    assert logs["dims"].sum() < 0.9 * logs["dcos"].sum() * D
    assert knn.recall(ids, gi, 10).mean() >= 0.7


def test_uneven_k_and_nprobe(setup):
    X, Q, _, index = setup
    K = np.array([1, 10, 3, 7, 10, 2, 5, 9, 4, 6, 8, 1])
    npb = np.array([1, 2, 3, 4, 5, 6, 7, 8, 16, 20, 2, 3])
    ids, d2 = ivf.search(index, Q, K, npb, 8)
    for qi in range(len(Q)):
        a, b = ivf.search(index, Q[qi:qi + 1], int(K[qi]), int(npb[qi]), 8)
        assert np.array_equal(ids[qi, :K[qi]], a[0]) and np.all(ids[qi, K[qi]:] == -1)
        assert np.all(np.isinf(d2[qi, K[qi]:]))


def test_round_starts_fill_then_schedule():
    rs = ivf.round_starts
    # lists of sizes 5, 7, 3, 4; K = 3, no fill minimum, no growth cap: fill [0,3), rest of
    # list 0, then each list
    assert rs(np.array([5, 7, 3, 4]), 3, "per_rank", 0, 0) == [0, 3, 5, 12, 15, 19]
    # K = 6 crosses into list 1: fill [0,6), then the rest of list 1
    assert rs(np.array([5, 7, 3, 4]), 6, "per_rank", 0, 0) == [0, 6, 12, 15, 19]
    # doubling: ranks end after lists 1, 2, 4 -> positions 5, 12, 19
    assert rs(np.array([5, 7, 3, 4]), 3, "doubling", 0, 0) == [0, 3, 5, 12, 19]
    # K larger than everything: one round
    assert rs(np.array([2, 2]), 10, "per_rank", 0, 0) == [0, 4]


def test_round_starts_fill_minimum_and_growth_cap():
    rs = ivf.round_starts
    sizes = np.array([5, 7, 3, 4])
    # growth 1: a round holds at most as many candidates as came before it
    #   3 -> min(cut 5, 6) = 5 -> min(12, 10) = 10 -> min(12, 20) = 12 -> 15 -> 19
    assert rs(sizes, 3, "per_rank", 0, 1) == [0, 3, 5, 10, 12, 15, 19]
    #   2 -> min(5, 4) = 4 -> min(5, 8) = 5 -> 10 -> 12 -> 15 -> 19
    assert rs(sizes, 2, "per_rank", 0, 1) == [0, 2, 4, 5, 10, 12, 15, 19]
    # doubling cuts 5, 12, 19 with growth 2: 1 -> min(5, 3) = 3 -> min(5, 9) = 5 -> 12 -> 19
    assert rs(sizes, 1, "doubling", 0, 2) == [0, 1, 3, 5, 12, 19]
    # a fill minimum of 8 makes the first round [0, 8), then the cuts after 8
    assert rs(sizes, 3, "per_rank", 8, 0) == [0, 8, 12, 15, 19]
    # the defaults (at least 32 in the first round) take all 19 candidates at once
    assert rs(sizes, 3, "per_rank") == [0, 19]
    # nothing to scan
    assert rs(np.array([0, 0]), 3, "per_rank") == [0]


def test_round_starts_whole_schedule():
    rs = ivf.round_starts
    sizes = np.array([5, 7, 3, 4])
    # no cut at a list end: the fill round, then everything else
    assert rs(sizes, 3, "whole", 0, 0) == [0, 3, 19]
    # growth 1 alone cuts the rest: 3 -> 6 -> 12 -> 19
    assert rs(sizes, 3, "whole", 0, 1) == [0, 3, 6, 12, 19]
    # one probed list: the same cuts as per-rank and doubling
    for g in (0, 1, 4):
        assert rs(np.array([40]), 3, "whole", 8, g) == rs(np.array([40]), 3, "per_rank", 8, g) == \
            rs(np.array([40]), 3, "doubling", 8, g)
    # two probed lists: the same cuts as doubling with the rank-1 cut taken away
    assert rs(np.array([20, 30]), 3, "doubling", 8, 0) == [0, 8, 20, 50]
    assert rs(np.array([20, 30]), 3, "whole", 8, 0) == [0, 8, 50]


def test_round_bounds():
    assert ivf.round_bounds(8, "whole") == [(0, 8)]
    assert ivf.round_bounds(8, "doubling") == [(0, 1), (1, 2), (2, 4), (4, 8)]
    assert ivf.round_bounds(6, "doubling") == [(0, 1), (1, 2), (2, 4), (4, 6)]
    assert ivf.round_bounds(3, "per_rank") == [(0, 1), (1, 2), (2, 3)]
    assert list(ivf.tested_dims(10, 3)) == [3, 6, 9]
    assert list(ivf.tested_dims(8, 4)) == [4]


def test_low_precision_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 50, [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_bf16(x), ref)
    ref16 = torch.from_numpy(x.astype(np.float32)).to(torch.float16).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_f16(x), ref16)


def test_low_precision_index_search(setup):
    X, Q, init, _ = setup
    pairs = workloads.calibration_pairs(N, 20000, seed=21)
    idx = ivf.build(X, NLIST, init, pairs, store=lambda y: lowp.store(y, "bf16"))
    assert 0 < idx.delta < 0.05
    ids, d2 = ivf.search(idx, Q, 10, 8, 8)
    for qi in range(len(Q)):
        v = ids[qi] >= 0
        exact = np.sum((X[ids[qi][v]].astype(np.float64) - Q[qi]) ** 2, axis=1)
        np.testing.assert_allclose(d2[qi][v], exact, rtol=1e-12)  # reranked with exact rows
    gi, _ = knn.brute_force(X, Q, 10)
    assert knn.recall(ids, gi, 10).mean() >= 0.7


def test_vectorised_round_on_hand_worked_cases():
    """The vectorised round scan reproduces the hand-worked Algorithm 1 cases."""
    from test_oracle_dco import EPS, LAM, _cases
    for case in _cases():
        dd, r, o, acc, dis, dexit = case.values
        index = ivf.Index(np.zeros(4), np.eye(4), LAM, EPS, np.zeros((1, 4)),
                          np.array([0, 1]), np.array([0]), o[None, :])
        hd = np.array([r * r]) if np.isfinite(r) else np.zeros(0)
        hi = np.array([10 ** 9]) if np.isfinite(r) else np.zeros(0, np.int64)
        d2, kept, exit_d, _, _ = ivf._scan_round(index, np.zeros(4), np.array([0]), hd, hi, 1, dd,
                                                 "dade", ivf.tested_dims(4, dd))
        assert int(exit_d[0]) == dexit, case.id
        assert (len(kept) == 1) == acc, case.id
        if acc:
            assert abs(d2[0] - dis * dis) <= 1e-12 * dis * dis


def test_keep_rule_breaks_distance_ties_by_id():
    """Two identical rows: once the heap holds id 0 (sequential, or the K = 1 fill round of
    per-rank), the later id ties with r and is not kept; the result is id 0 either way."""
    X = np.array([[1.0, 0.0], [1.0, 0.0], [3.0, 0.0]])
    index = ivf.Index(np.zeros(2), np.eye(2), np.array([1.0, 1.0]), np.zeros(2),
                      np.zeros((1, 2)), np.array([0, 3]), np.array([0, 1, 2]), X)
    q = np.zeros((1, 2))
    ids, d2, logs = ivf.search(index, q, 1, 1, 1, mode="exact", schedule="sequential", log=True)
    assert ids[0, 0] == 0 and logs["accepted"][0] == 1
    ids, d2, logs = ivf.search(index, q, 1, 1, 1, mode="exact", schedule="per_rank", log=True,
                               fill_min=0, growth=0)
    assert ids[0, 0] == 0 and logs["accepted"][0] == 1
    # with the default fill minimum all three rows fill the heap in one round; id 0 wins the tie
    ids, d2, logs = ivf.search(index, q, 1, 1, 1, mode="exact", schedule="per_rank", log=True)
    assert ids[0, 0] == 0 and logs["accepted"][0] == 3


@pytest.mark.parametrize("rerank", ["all", "lazy"])
@pytest.mark.parametrize("delta", [0.0, 0.01, 1e9])
def test_rerank_rule_with_exact_store_changes_nothing(setup, delta, rerank):
    """With stored coordinates equal to the exact ones, the rerank rule (K smallest reranked,
    the rest only within (1 + delta) of the K-th exact distance) keeps exactly the results of
    the plain index for any delta >= 0: a candidate it skips is farther than the final K-th."""
    import dataclasses
    X, Q, _, index = setup
    lp = dataclasses.replace(index, Y_exact=index.Y, delta=delta)
    for schedule in ("per_rank", "doubling"):
        a_i, a_d = ivf.search(index, Q, 10, 6, 8, schedule=schedule)
        b_i, b_d = ivf.search(lp, Q, 10, 6, 8, schedule=schedule, rerank=rerank)
        assert np.array_equal(a_i, b_i)
        np.testing.assert_allclose(a_d, b_d, rtol=1e-12)


def test_rerank_rule_reranks_few_when_heap_empty(setup):
    """Round 0 (empty heap) queues every survivor but reranks only the K smallest and those
    within the bound -- far fewer than the list."""
    X, Q, init, _ = setup
    pairs = workloads.calibration_pairs(N, 20000, seed=21)
    idx = ivf.build(X, NLIST, init, pairs, store=lambda y: lowp.store(y, "bf16"))
    calls = []
    orig = idx.Y_exact
    class Counting:
        def __getitem__(self, rows):
            calls.append(len(np.atleast_1d(rows)))
            return orig[rows]
    idx.Y_exact = Counting()
    ivf.search(idx, Q[:1], 10, 1, 8, rerank="lazy")
    list_len = max(np.diff(idx.offsets))
    assert 10 <= sum(calls) < list_len
    # the plain rule reranks every survivor of the round (the heap is empty: all of them)
    calls.clear()
    ivf.search(idx, Q[:1], 10, 1, 8, rerank="all", fill_min=0, growth=0)
    assert sum(calls) >= 10 and calls[0] == 10


def _two_list_index(stored, exact, n0, delta=0.1):
    """W = I index in 2-D: list 0 = ids [0, n0) (centroid near q = 0), list 1 = the rest."""
    Ys, Ye = np.asarray(stored, float), np.asarray(exact, float)
    return ivf.Index(np.zeros(2), np.eye(2), np.array([1.0, 1.0]), np.zeros(2),
                     np.array([[0.1, 0.0], [5.0, 5.0]]), np.array([0, n0, len(Ys)]), np.arange(len(Ys)),
                     Ys, Y_exact=Ye, delta=delta)


def _search2(index, nprobe, rerank="lazy"):
    """K = 2, first round = the first K candidates, then one round per list."""
    ids, d2 = ivf.search(index, np.zeros((1, 2)), 2, nprobe, 1, mode="exact", fill_min=0, growth=0,
                         rerank=rerank)
    return list(ids[0]), d2[0]


def test_rerank_rule_hand_worked_f_is_k_smallest():
    """K = 2, delta = 0.1, full-D DCOs, per-rank.  (stored S_D / exact S_D)
    list 0: id0 1.0/1.0, id1 1.44/1.44, id2 4.0/4.0; list 1: id3 1.45/1.09, id4 1.4641/1.04,
    id5 1.565/1.565.  Fill round {0, 1}: heap (1.0, 0), (1.44, 1).  Rest of list 0: id2 fails
    the gate 1.584.  List 1: all pass the gate; F = {3, 4} (two smallest stored) -> exact
    1.09, 1.04; b = 2nd of {1.0, 1.44, 1.09, 1.04} = 1.04, bound 1.144: id5 not reranked.
    Both of F kept -> heap (1.0, 0), (1.04, 4)."""
    index = _two_list_index([[1, 0], [0, 1.2], [2, 0], [1.2, 0.1], [0, 1.21], [1.25, 0.05]],
                            [[1, 0], [0, 1.2], [2, 0], [1.0, 0.3], [1.0, 0.2], [1.25, 0.05]], 3)
    ids, d2 = _search2(index, 1)
    assert ids == [0, 1]
    ids, d2 = _search2(index, 2)
    assert ids == [0, 4]
    np.testing.assert_allclose(d2, [1.0, 1.04], rtol=1e-12)
    # plain rule: every gated survivor reranked (1.09, 1.04, 1.565); the keep rule drops 1.565
    assert _search2(index, 2, "all")[0] == [0, 4]


def test_rerank_rule_hand_worked_rest_within_bound():
    """As above but list 1: id3 1.45/1.5025, id4 1.4641/1.5625, id5 1.4741/1.21.
    F = {3, 4} -> exact 1.5025, 1.5625; b = 2nd of {1.0, 1.44, 1.5025, 1.5625} = 1.44,
    bound 1.584 >= 1.4741: id5 reranked (1.21) and kept; F's exact values exceed r^2 = 1.44.
    Heap -> (1.0, 0), (1.21, 5)."""
    index = _two_list_index([[1, 0], [0, 1.2], [2, 0], [1.2, 0.1], [0, 1.21], [1.21, 0.1]],
                            [[1, 0], [0, 1.2], [2, 0], [1.2, 0.25], [0, 1.25], [1.1, 0]], 3)
    ids, d2 = _search2(index, 2)
    assert ids == [0, 5]
    np.testing.assert_allclose(d2, [1.0, 1.21], rtol=1e-12)
    assert _search2(index, 2, "all")[0] == [0, 5]


def test_rerank_rule_hand_worked_bound_uses_heap():
    """Heap after list 0: (1.0, 0), (1.21, 1).  List 1: id2 stored (0, 1.03) 1.0609 / exact
    (1.01, 0) 1.0201; id3 (0, 1.04) 1.0816 / (1.02, 0) 1.0404; id4 (0, 1.065) 1.134225 /
    (1.005, 0) 1.010025.  Gate 1.331 passes all; F = {2, 3}; b = 2nd of {1.0, 1.21, 1.0201,
    1.0404} = 1.0201, bound 1.12211 < 1.134225: id4 is NOT reranked (b computed from F alone
    would be 1.0404 and let it in).  Heap -> (1.0, 0), (1.0201, 2)."""
    index = _two_list_index([[1, 0], [1.1, 0], [0, 1.03], [0, 1.04], [0, 1.065]],
                            [[1, 0], [1.1, 0], [1.01, 0], [1.02, 0], [1.005, 0]], 2)
    ids, d2 = _search2(index, 2)
    assert ids == [0, 2]
    np.testing.assert_allclose(d2, [1.0, 1.0201], rtol=1e-12)
    # the plain rule reranks id4 too (exact 1.010025 < 1.0201): the two rules differ here because
    # id4's stored-precision error (1.134225 / 1.010025 - 1 = 0.123) exceeds delta = 0.1
    ids, d2 = _search2(index, 2, "all")
    assert ids == [0, 4]
    np.testing.assert_allclose(d2, [1.0, 1.010025], rtol=1e-12)
