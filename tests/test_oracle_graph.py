"""Pins of the graph-search oracle (oracle/graph.py) against what the definitions fix: the kNN
graph against brute force (oracle/knn.py, a separate implementation), the medoid's minimality,
a beam that sees every object returning the exact KNN, the FDScanning beam returning the exact
top-K of what it visited, and DADE with tests that never reject reducing to FDScanning."""
import dataclasses

import numpy as np
import pytest

from oracle import graph, ivf, knn, lowp

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def gaussian(n, d, seed, centres=4):
    rng = np.random.default_rng(seed)
    C = rng.normal(0, 3, (centres, d))
    return (C[rng.integers(0, centres, n)] + rng.normal(0, 1, (n, d)) * np.linspace(2, 0.2, d)).astype(np.float32)


def small_index(n=400, d=16, nlist=6, seed=0, store=None):
    X = gaussian(n, d, seed)
    rng = np.random.default_rng(seed + 1)
    init = rng.choice(n, nlist, replace=False)
    pairs = np.stack([rng.integers(0, n, 4000), rng.integers(0, n, 4000)], 1)
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    st = None if store is None else (lambda y: lowp.store(y, store))
    return X, ivf.build(X, nlist, init, pairs, p_s=0.1, iters=5, store=st)


def test_knn_graph_over_all_lists_is_brute_force():
    X, oi = small_index()
    G = graph.build_knn_graph(oi, X, degree=8, nprobe=oi.nlist)
    bf, _ = knn.brute_force(X, X, 9)
    for i in range(len(X)):
        assert G[i].tolist() == [v for v in bf[i].tolist() if v != i][:8], i


def test_medoids_are_members_nearest_their_centroid():
    X, oi = small_index()
    med = graph.list_medoids(oi, X)
    for l in range(oi.nlist):
        members = oi.ids[oi.offsets[l]:oi.offsets[l + 1]]
        assert med[l] in members
        dm = np.sum((X[med[l]].astype(np.float64) - oi.centroids[l]) ** 2)
        for m in members:
            assert np.sum((X[m].astype(np.float64) - oi.centroids[l]) ** 2) >= dm


@pytest.mark.parametrize("mode", ["full_d", "dade"])
def test_beam_over_a_complete_graph_is_exact_knn(mode):
    """Every object is a neighbour of every seed and ef >= n: the pool ends holding every object
    that was not rejected; in FDScanning mode that is all of them, so the result is the KNN."""
    X, oi = small_index(n=60, nlist=3)
    n = len(X)
    G = np.array([[j for j in range(n) if j != i] for i in range(n)])
    med = graph.list_medoids(oi, X)
    Q = gaussian(12, X.shape[1], 9)
    ids, d2, logs = graph.search(oi, G, med, Q, 10, ef=n, n_entry=oi.nlist, delta_d=4, mode=mode, log=True)
    bf_i, bf_d = knn.brute_force(X, Q, 10)
    if mode == "full_d":
        np.testing.assert_array_equal(ids, bf_i)
        np.testing.assert_allclose(d2, bf_d, rtol=1e-12)
    assert np.all(logs["visited"] == n)
    # returned distances are exact whatever the mode
    for q in range(len(Q)):
        ex = np.sum((X[ids[q]].astype(np.float64) - Q[q].astype(np.float64)) ** 2, axis=1)
        np.testing.assert_allclose(d2[q], ex, rtol=1e-12)


@pytest.mark.parametrize("ef", [4, 10, 24])
def test_full_d_beam_returns_the_top_k_of_what_it_visited(ef):
    """An object dropped at any step was farther than that step's r, which only shrinks, so the
    FDScanning pool ends as the ef nearest of the visited set and the result as its K nearest."""
    X, oi = small_index(seed=3)
    G = graph.build_knn_graph(oi, X, degree=6, nprobe=2)
    med = graph.list_medoids(oi, X)
    Q = gaussian(20, X.shape[1], 11)
    K = min(4, ef)
    ids, d2, logs = graph.search(oi, G, med, Q, K, ef=ef, n_entry=2, delta_d=4, mode="full_d", log=True)
    for q in range(len(Q)):
        vis = logs["visited_ids"][q]
        bi, bd = knn.brute_force(X[vis], Q[q:q + 1], K)
        assert ids[q].tolist() == vis[bi[0]].tolist(), q
        np.testing.assert_allclose(d2[q], bd[0], rtol=1e-12)


def test_dade_without_rejections_is_full_d():
    X, oi = small_index(seed=5)
    G = graph.build_knn_graph(oi, X, degree=6, nprobe=2)
    med = graph.list_medoids(oi, X)
    Q = gaussian(15, X.shape[1], 13)
    never = dataclasses.replace(oi, eps=np.full_like(oi.eps, np.inf))
    a = graph.search(never, G, med, Q, 5, ef=12, n_entry=2, delta_d=4, mode="dade", log=True)
    b = graph.search(oi, G, med, Q, 5, ef=12, n_entry=2, delta_d=4, mode="full_d", log=True)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    # the calibrated tests do reject and read fewer dimensions
    c = graph.search(oi, G, med, Q, 5, ef=12, n_entry=2, delta_d=4, mode="dade", log=True)
    assert c[2]["dims"].sum() < b[2]["dims"].sum()


def test_low_precision_beam_returns_exact_distances():
    X, oi = small_index(seed=7, store="bf16")
    G = graph.build_knn_graph(oi, X, degree=6, nprobe=2)
    med = graph.list_medoids(oi, X)
    Q = gaussian(10, X.shape[1], 17)
    ids, d2, _ = graph.search(oi, G, med, Q, 5, ef=12, n_entry=2, delta_d=4, log=True)
    for q in range(len(Q)):
        v = ids[q] >= 0
        ex = np.sum((X[ids[q][v]].astype(np.float64) - Q[q].astype(np.float64)) ** 2, axis=1)
        np.testing.assert_allclose(d2[q][v], ex, rtol=1e-10)
        assert list(d2[q][v]) == sorted(d2[q][v])


def test_reverse_edges_link_back_nearest_first():
    """Every listed back link is a row that points here; each row keeps its forward list first;
    the back links are the nearest such rows (brute force over all in-links); no duplicates."""
    X, oi = small_index(seed=11)
    G = graph.build_knn_graph(oi, X, degree=4, nprobe=2)
    H = graph.add_reverse_edges(G, X, reverse=3)
    assert H.shape == (len(X), 7)
    Xd = X.astype(np.float64)
    for v in range(len(X)):
        row = [int(u) for u in H[v] if u >= 0]
        assert len(row) == len(set(row)) and v not in row
        assert row[:4] == [int(u) for u in G[v] if u >= 0]
        back = row[4:]
        pointing = [u for u in range(len(X)) if v in G[u] and u not in G[v]]
        assert set(back) <= set(pointing)
        want = sorted(pointing, key=lambda u: (np.sum((Xd[u] - Xd[v]) ** 2), u))[:3]
        assert back == want, v
    # every row that has an in-link can now be reached back from it
    assert sum((H >= 0).sum(1)) > sum((G >= 0).sum(1))


def test_second_entry_is_the_member_farthest_from_the_medoid():
    X, oi = small_index(seed=13)
    E = graph.list_entries(oi, X)
    med = graph.list_medoids(oi, X)
    Xd = X.astype(np.float64)
    for l in range(oi.nlist):
        members = oi.ids[oi.offsets[l]:oi.offsets[l + 1]]
        assert E[l, 0] == med[l]
        if len(members) < 2:
            assert E[l, 1] == -1
            continue
        far = max(members, key=lambda m: (np.sum((Xd[m] - Xd[med[l]]) ** 2), -m))
        assert E[l, 1] == far and E[l, 1] != E[l, 0]


def test_two_entries_per_list_reach_a_component_the_medoid_misses():
    """Two well-separated blobs in one list: the medoid sits in the larger blob; a query beside
    the smaller blob is only reached through the second entry point (a kNN graph has no edge
    between the blobs)."""
    rng = np.random.default_rng(3)
    A = rng.normal(0, 1, (60, 8))
    B = rng.normal(0, 1, (20, 8)) + 40.0
    X = np.concatenate([A, B]).astype(np.float32)
    pairs = np.stack([rng.integers(0, 80, 2000), rng.integers(0, 80, 2000)], 1)
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    oi = ivf.build(X, 1, np.array([0]), pairs, p_s=0.1, iters=1)
    G = graph.build_knn_graph(oi, X, degree=5, nprobe=1)
    q = (B[:1] + 0.1).astype(np.float32)
    gt, _ = knn.brute_force(X, q, 5)
    one, _, _ = graph.search(oi, G, graph.list_medoids(oi, X), q, 5, ef=8, n_entry=1, delta_d=4, mode="full_d")
    two, _, _ = graph.search(oi, G, graph.list_entries(oi, X), q, 5, ef=8, n_entry=1, delta_d=4, mode="full_d")
    assert not set(one[0]) & set(gt[0])
    assert set(two[0]) == set(gt[0])


def test_selection_on_a_line_keeps_one_neighbour_per_side():
    """Hand-worked: v at 0 with candidates at 1, 2, 3, -1, -2 (ids 1..5).  1 is kept first (ties
    with -1 at distance 1 go to the lower id); 2 and 3 are nearer 1 than 0; -1 is nearer 0 than 1
    and is kept; -2 is nearer -1."""
    X = np.array([[0.0], [1.0], [2.0], [3.0], [-1.0], [-2.0]])
    kept, margin = graph.select_neighbors(X, 0, [1, 2, 3, 4, 5], 4)
    assert kept == [1, 4]
    assert margin == 0.0   # the exact tie between ids 1 and 4, broken by id


def test_selection_keeps_a_candidate_equidistant_from_v_and_a_kept_neighbour():
    """Only a strictly closer kept neighbour prunes: e = (1, 2) is at squared distance 5 from both
    v = (0, 0) and the kept r = (2, 0), so it stays; (3, 0) is nearer r and goes."""
    X = np.array([[0.0, 0.0], [2.0, 0.0], [1.0, 2.0], [3.0, 0.0]])
    kept, margin = graph.select_neighbors(X, 0, [1, 2, 3], 3)
    assert kept == [1, 2]
    assert margin == 0.0


def test_selection_of_mutually_far_candidates_keeps_the_nearest_m():
    """Candidates on distinct axes at lengths 1.0 .. 1.4: d(e_i, e_j)^2 = s_i^2 + s_j^2 exceeds
    both s_i^2 and s_j^2, so nothing is pruned and the first M by distance are kept."""
    s = np.array([1.3, 1.0, 1.4, 1.1, 1.2])
    X = np.zeros((6, 5))
    X[1:, :] = np.diag(s)
    assert graph.select_neighbors(X, 0, [1, 2, 3, 4, 5], 10)[0] == [2, 4, 5, 1, 3]
    assert graph.select_neighbors(X, 0, [1, 2, 3, 4, 5], 3)[0] == [2, 4, 5]
    assert graph.select_neighbors(X, 0, [5, 4, 3, 2, 1], 1)[0] == [2]


def test_selection_links_a_far_blob_that_the_nearest_rows_do_not():
    """v = (0, 0) with four collinear rows to its right and two rows 5 away above: the nearest 2
    are both to the right, while the heuristic keeps the first row to the right (it prunes the
    other three) and the nearer row above (squared distance 25 from v, 25.01 from (0.1, 0))."""
    X = np.array([[0.0, 0.0], [0.1, 0.0], [0.2, 0.0], [0.3, 0.0], [0.4, 0.0], [0.0, 5.0], [0.1, 5.0]])
    kept, _ = graph.select_neighbors(X, 0, [1, 2, 3, 4, 5, 6], 2)
    assert kept == [1, 5]
    bf, _ = knn.brute_force(X.astype(np.float32), X[:1].astype(np.float32), 3)
    assert [v for v in bf[0].tolist() if v != 0][:2] == [1, 2]


def test_graph_with_selection_over_all_lists():
    """With every list probed, the candidates are the brute-force nearest rows, and each row's
    out-neighbours are what the heuristic keeps among them; fewer than degree where it prunes."""
    X, oi = small_index(seed=19)
    G, info = graph.build_knn_graph(oi, X, degree=6, nprobe=oi.nlist, candidates=20, log=True)
    bf, _ = knn.brute_force(X, X, 22)
    pruned = 0
    for i in range(len(X)):
        cand = [v for v in bf[i].tolist() if v != i][:20]
        kept, _ = graph.select_neighbors(X, i, cand, 6)
        assert G[i].tolist() == kept + [-1] * (6 - len(kept)), i
        pruned += 6 - len(kept)
        # every kept pair satisfies the rule: no earlier kept row is strictly closer to a later one
        Xd = X.astype(np.float64)
        for a in range(len(kept)):
            for b in range(a):
                assert np.sum((Xd[kept[a]] - Xd[kept[b]]) ** 2) >= np.sum((Xd[kept[a]] - Xd[i]) ** 2)
    assert pruned > 0 and np.all(info["boundary"] >= 0) and np.all(info["select"] >= 0)
