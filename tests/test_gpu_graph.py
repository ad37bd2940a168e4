"""Graph search on the GPU (dade_graph_build / dade_graph_search) against the oracle
(oracle/graph.py): the kNN graph and the entry points the library builds, then beam searches in
DADE and FDScanning modes, FP32 and BF16 stores, run by the oracle on the library's own graph
(exported as row ids) and compared element by element, near ties excused by their logged margins."""
import numpy as np
import pytest

from oracle import graph, ivf
from paper_2411_17229_amd import dade, workloads
from gpu_helpers import EXCUSE_TOL, artifacts, compare, integer_index, oracle_graph, oracle_index, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEG, REV, NPROBE_BUILD = 16, 8, 4


def _setup(store):
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n_queries=200)
    oi, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha, store=store)
    Xd = torch.from_numpy(X).cuda()
    gi = dade.dade_import(artifacts(oi), Xd, store=store or "f32")
    dade.dade_graph_build(gi, degree=DEG, reverse=REV, nprobe=NPROBE_BUILD)
    nb, en = dade.dade_graph_export(gi)
    return dict(w=w, X=X, Q=Q, Qd=torch.from_numpy(Q).cuda(), oi=oi, gi=gi, nb=nb, en=en)


@pytest.fixture(scope="module")
def f32():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return _setup(None)


@pytest.fixture(scope="module")
def bf16():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return _setup("bf16")


def test_graph_build_matches_oracle(f32):
    """Sampled rows: the same neighbour distances as the oracle's FDScanning kNN (ids may swap only
    between equal distances)."""
    X, oi, nb = f32["X"], f32["oi"], f32["nb"]
    rows = np.sort(np.random.default_rng(0).choice(len(X), 300, replace=False))
    o_nb = graph.build_knn_graph(oi, X, DEG, NPROBE_BUILD, rows=rows)
    Xd = X.astype(np.float64)
    assert nb.shape == (len(X), DEG + REV)
    for i, r in enumerate(rows):
        fwd = nb[r, :DEG]
        assert np.all(fwd >= 0) and r not in nb[r]
        dg = np.sum((Xd[fwd] - Xd[r]) ** 2, axis=1)
        do = np.sum((Xd[o_nb[i]] - Xd[r]) ** 2, axis=1)
        np.testing.assert_allclose(dg, do, rtol=1e-5, err_msg=f"row {r}")
        assert np.all(np.diff(dg) >= -1e-5 * dg[1:]), r
    # back links: the oracle's rule applied to the library's forward lists
    H = graph.add_reverse_edges(nb[:, :DEG], X, REV)
    for r in rows:
        got = [u for u in nb[r, DEG:] if u >= 0]
        want = [u for u in H[r, DEG:] if u >= 0]
        assert len(got) == len(want), r
        dg = np.sum((Xd[got] - Xd[r]) ** 2, axis=1)
        dw = np.sum((Xd[want] - Xd[r]) ** 2, axis=1)
        np.testing.assert_allclose(dg, dw, rtol=1e-12, err_msg=f"row {r}")


SEL_DEG, SEL_REV, SEL_CAND = 16, 16, 48


@pytest.fixture(scope="module")
def f32_sel():
    """The 20k x 128 index with HNSW neighbour selection over 48 candidates: its forward lists
    (a build with no back links) and its full rows (16 + 16 wide)."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    env = _setup(None)
    dade.dade_graph_build(env["gi"], degree=SEL_DEG, reverse=0, nprobe=NPROBE_BUILD, candidates=SEL_CAND)
    fwd, _ = dade.dade_graph_export(env["gi"])
    dade.dade_graph_build(env["gi"], degree=SEL_DEG, reverse=SEL_REV, nprobe=NPROBE_BUILD, candidates=SEL_CAND)
    env["nb"], env["en"] = dade.dade_graph_export(env["gi"])
    env["fwd"] = fwd
    return env


def test_graph_build_with_selection_matches_oracle(f32_sel):
    """Sampled rows: the out-neighbours are what the oracle's heuristic keeps among the oracle's
    FDScanning candidates, id for id and in order, wherever neither the candidate boundary nor a
    decision is a near tie; the full rows are the forward lists followed by the oracle's back
    links over the library's forward lists."""
    X, oi, fwd, nb = f32_sel["X"], f32_sel["oi"], f32_sel["fwd"], f32_sel["nb"]
    assert fwd.shape == (len(X), SEL_DEG) and nb.shape == (len(X), SEL_DEG + SEL_REV)
    rows = np.sort(np.random.default_rng(1).choice(len(X), 300, replace=False))
    o_nb, info = graph.build_knn_graph(oi, X, SEL_DEG, NPROBE_BUILD, rows=rows, candidates=SEL_CAND, log=True)
    clear = (info["boundary"] > 1e-4) & (info["select"] > 1e-9)
    assert clear.mean() > 0.9
    for i, r in enumerate(rows):
        got = [int(u) for u in fwd[r] if u >= 0]
        assert r not in got and len(set(got)) == len(got)
        assert all(u < 0 for u in fwd[r, len(got):]), r   # kept ones first, then padding
        if clear[i]:
            assert got == [int(u) for u in o_nb[i] if u >= 0], f"row {r}"
    pruned = (fwd < 0).sum()
    assert pruned > 0   # the heuristic does prune on this workload
    H = graph.add_reverse_edges(fwd, X, SEL_REV)
    np.testing.assert_array_equal(nb[rows], H[rows])


@pytest.mark.parametrize("mode", ["dade", "full_d"])
def test_graph_search_with_selection_matches_oracle(f32_sel, mode):
    st, _ = run_parity(f32_sel, mode)
    assert st[:, 2].max() <= 2 * 48


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_graph_exact_integer_inputs_match_exactly(store):
    """Where FP32 is exact (integer coordinates, W = I, dyadic thresholds, duplicate rows: every
    distance and threshold product is exact, every tie is broken by id), nothing is excused: the
    selected graph's forward lists equal the oracle's, and every query's ids, distances (bit for
    bit), DCOs, dimensions read, expansions and visits equal the oracle's beam on the library's
    graph, in DADE and FDScanning modes."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    X, Q, oi = integer_index(store, 2.0 ** -10)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda(), store=store)
    Qd = torch.from_numpy(Q).cuda()
    deg, rev, cand = 8, 4, 24
    dade.dade_graph_build(gi, degree=deg, reverse=0, nprobe=oi.nlist, candidates=cand)
    fwd, _ = dade.dade_graph_export(gi)
    rows = np.arange(0, len(X), 10)
    o_fwd = graph.build_knn_graph(oi, X, deg, oi.nlist, rows=rows, candidates=cand)
    np.testing.assert_array_equal(fwd[rows], o_fwd)
    dade.dade_graph_build(gi, degree=deg, reverse=rev, nprobe=oi.nlist, candidates=cand)
    nb, en = dade.dade_graph_export(gi)
    np.testing.assert_array_equal(nb, graph.add_reverse_edges(fwd, X, rev))
    np.testing.assert_array_equal(en, graph.list_entries(oi, X))
    for mode in ("dade", "full_d"):
        for K, ef, n_entry in ((5, 16, 2), (10, 32, 1), (1, 8, 4)):
            stats = torch.zeros((len(Q), 4), dtype=torch.int64, device="cuda")
            ids, d2 = dade.dade_graph_search(gi, Qd, K, ef, n_entry=n_entry, delta_d=8, mode=mode, stats=stats)
            torch.cuda.synchronize()
            o_ids, o_d2, logs = graph.search(oi, nb, en, Q, K, ef, n_entry, 8, mode=mode, log=True)
            assert np.array_equal(to_np(ids), o_ids), (mode, K, ef, n_entry)
            assert np.array_equal(to_np(d2).astype(np.float64), o_d2), (mode, K, ef, n_entry)
            st = to_np(stats)
            for j, key in enumerate(("dcos", "dims", "expansions", "visited")):
                np.testing.assert_array_equal(st[:, j], logs[key].astype(np.int64), err_msg=f"{mode} {key}")
    gi.close()


def test_entry_points_are_medoid_and_farthest_member(f32):
    X, oi, en = f32["X"], f32["oi"], f32["en"]
    assert en.shape == (oi.nlist, 2)
    med = graph.list_medoids(oi, X)
    Xd = X.astype(np.float64)
    for l in range(oi.nlist):
        members = oi.ids[oi.offsets[l]:oi.offsets[l + 1]]
        assert en[l, 0] in members and en[l, 1] in members and en[l, 0] != en[l, 1]
        d_g = np.sum((Xd[en[l, 0]] - oi.centroids[l]) ** 2)
        d_o = np.sum((Xd[med[l]] - oi.centroids[l]) ** 2)
        assert abs(d_g - d_o) <= 1e-5 * d_o, l
        # the second entry: the member farthest from the library's medoid
        far = np.sum((Xd[members] - Xd[en[l, 0]]) ** 2, axis=1).max()
        assert abs(np.sum((Xd[en[l, 1]] - Xd[en[l, 0]]) ** 2) - far) <= 1e-5 * far, l


def run_parity(env, mode, K=10, ef=48, n_entry=4, max_iters=0, dd=32):
    nq = len(env["Q"])
    stats = torch.zeros((nq, 4), dtype=torch.int64, device="cuda")
    ids, d2 = dade.dade_graph_search(env["gi"], env["Qd"], K, ef, n_entry=n_entry, max_iters=max_iters,
                                     delta_d=dd, mode=mode, stats=stats)
    torch.cuda.synchronize()
    ids, d2, st = to_np(ids), to_np(d2), to_np(stats)
    o = oracle_graph(env["oi"], env["nb"], env["en"], env["Q"], K, ef, n_entry, dd, mode=mode, max_iters=max_iters)
    logs = o.logs
    compare(o, ids, d2, env["X"], env["Q"], K)
    # queries without a near tie follow the same trajectory: the same DCOs, steps and visits
    same = (logs["min_margin"] > EXCUSE_TOL) & (logs["probe_gap"] > EXCUSE_TOL)
    assert same.mean() > 0.9
    np.testing.assert_array_equal(st[same, 0], logs["dcos"][same])
    np.testing.assert_array_equal(st[same, 1], logs["dims"][same])
    np.testing.assert_array_equal(st[same, 2], logs["expansions"][same])
    np.testing.assert_array_equal(st[same, 3], logs["visited"][same])
    return st, logs


@pytest.mark.parametrize("mode", ["dade", "full_d"])
def test_graph_search_matches_oracle_f32(f32, mode):
    st, _ = run_parity(f32, mode)
    if mode == "dade":   # some tests exit early (a graph's candidates are near ones, so fewer than in IVF)
        assert st[:, 1].sum() < st[:, 0].sum() * f32["w"].dim


@pytest.mark.parametrize("ef,n_entry,max_iters,dd", [(10, 1, 0, 8), (64, 8, 40, 16), (32, 2, 0, 64), (8, 8, 0, 16)])
def test_graph_search_parameters(f32, ef, n_entry, max_iters, dd):
    """Includes 2 n_entry > ef: the seed merge keeps only the ef nearest of 16 seeds."""
    run_parity(f32, "dade", K=min(10, ef), ef=ef, n_entry=n_entry, max_iters=max_iters, dd=dd)


def test_graph_search_matches_oracle_bf16(bf16):
    run_parity(bf16, "dade")


def test_graph_search_batch_invariance(f32):
    ids_b, d2_b = dade.dade_graph_search(f32["gi"], f32["Qd"], 10, 48, n_entry=4)
    ids_b, d2_b = to_np(ids_b), to_np(d2_b)
    for qi in (0, 77, 199):
        i1, d1 = dade.dade_graph_search(f32["gi"], f32["Qd"][qi:qi + 1].contiguous(), 10, 48, n_entry=4)
        assert np.array_equal(to_np(i1)[0], ids_b[qi]) and np.array_equal(to_np(d1)[0].view(np.uint32),
                                                                         d2_b[qi].view(np.uint32))


def test_graph_argument_errors(f32):
    gi, Qd = f32["gi"], f32["Qd"]
    for kw in (dict(k=10, ef=65), dict(k=20, ef=10), dict(k=10, ef=32, delta_d=12), dict(k=10, ef=32, n_entry=0),
               dict(k=10, ef=32, n_entry=33), dict(k=10, ef=64, max_iters=300)):
        k, ef = kw.pop("k"), kw.pop("ef")
        with pytest.raises(dade.DadeError):
            dade.dade_graph_search(gi, Qd, k, ef, **kw)
    other = dade.dade_import(artifacts(f32["oi"]), torch.from_numpy(f32["X"]).cuda())
    with pytest.raises(dade.DadeError):   # no graph yet
        dade.dade_graph_search(other, Qd, 10, 32)
    other.close()


def test_graph_build_rejects_indexes_above_its_limit():
    """Builds above 20,000 rows are refused before any device work (the check is on the host)."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    w = workloads.WORKLOADS["small-20k-d128"]
    X = np.concatenate([workloads.make(w)[0], workloads.make(w)[0][:10]])
    Xd = torch.from_numpy(X).cuda()
    gi = dade.dade_build_index(Xd, 16, kmeans_iters=1)
    dade.dade_rotate(gi)
    with pytest.raises(dade.DadeError, match="not supported"):
        dade.dade_graph_build(gi, degree=8, reverse=0, nprobe=2)
    gi.close()
