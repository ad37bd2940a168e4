"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs (the 20k x 128 workload and smaller edge-case inputs).  The oracle builds the index;
its artifacts are imported into the library so both scan identical lists."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from gpu_helpers import (artifacts, compare, oracle_ivf, exact_d2, gpu_search, integer_index, oracle_index,
                         to_np)
from oracle import estimator, ivf, knn, pca
from paper_2411_17229_amd import dade, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def small():
    _need_gpu()
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w)
    oi, init, pairs = oracle_index(X, w.nlist, w.seed, alpha=w.alpha)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    gi = dade.dade_import(artifacts(oi), Xd)
    return dict(w=w, X=X, Q=Q, oi=oi, init=init, pairs=pairs, Xd=Xd, Qd=Qd, gi=gi)


@pytest.mark.parametrize("schedule", ["per_rank", "doubling"])
def test_full_d_matches_oracle(small, schedule):
    w, oi = small["w"], small["oi"]
    o = oracle_ivf(oi, small["Q"], w.k, w.nprobe, w.delta_d, mode="exact")
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, mode="full_d", schedule=schedule)
    compare(o, g_ids, g_d2, small["X"], small["Q"], w.k)


@pytest.mark.parametrize("schedule", ["per_rank", "doubling", "whole"])
def test_dade_matches_oracle(small, schedule):
    w, oi = small["w"], small["oi"]
    o = oracle_ivf(oi, small["Q"], w.k, w.nprobe, w.delta_d, schedule=schedule)
    logs = o.logs
    stats = torch.zeros((w.n_queries, 4), dtype=torch.int64, device="cuda")
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, delta_d=w.delta_d, schedule=schedule,
                             stats=stats)
    compare(o, g_ids, g_d2, small["X"], small["Q"], w.k)
    st = to_np(stats)
    # DCO counts are exact; dimensions read match the oracle's Algorithm 1 logs up to
    # near-tie decisions
    np.testing.assert_array_equal(st[:, 0], logs["dcos"].astype(np.int64))
    rel = np.abs(st[:, 1] - logs["dims"]) / logs["dims"]
    assert np.median(rel) == 0.0 and rel.max() < 0.02
    assert st[:, 1].sum() < 0.8 * st[:, 0].sum() * w.dim   # the test really exits early


@pytest.mark.parametrize("fill_min,growth,schedule", [(0, 0, "per_rank"), (0, 1, "per_rank"), (8, 2, "doubling"),
                                                      (200, 4, "per_rank"), (0, 2, "whole")])
def test_round_size_options(small, fill_min, growth, schedule):
    """First-round minimum and growth cap: the same round cuts as the oracle's, so DCO counts
    agree exactly and results agree up to near ties."""
    w, oi = small["w"], small["oi"]
    o = oracle_ivf(oi, small["Q"], w.k, w.nprobe, w.delta_d, schedule=schedule,
                   fill_min=fill_min, growth=growth)
    logs = o.logs
    stats = torch.zeros((w.n_queries, 4), dtype=torch.int64, device="cuda")
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, delta_d=w.delta_d, schedule=schedule,
                             stats=stats, fill_min=fill_min, growth=growth)
    compare(o, g_ids, g_d2, small["X"], small["Q"], w.k)
    st = to_np(stats)
    np.testing.assert_array_equal(st[:, 0], logs["dcos"].astype(np.int64))
    rel = np.abs(st[:, 1] - logs["dims"]) / logs["dims"]
    assert np.median(rel) == 0.0 and rel.max() < 0.02


@pytest.mark.parametrize("schedule", ["per_rank", "doubling"])
def test_graph_replays_match_eager(small, schedule):
    """The captured launch sequence, replayed several times with eager searches and
    synchronisations in between, gives the eager result bit for bit every time."""
    w, gi, Qd = small["w"], small["gi"], small["Qd"]
    kw = dict(delta_d=w.delta_d, schedule=schedule)
    ref_i, ref_d = gpu_search(gi, Qd, w.k, w.nprobe, use_graph=False, **kw)
    out_i = torch.empty((w.n_queries, w.k), dtype=torch.int64, device="cuda")
    out_d = torch.empty((w.n_queries, w.k), dtype=torch.float32, device="cuda")
    for _ in range(4):
        out_i.fill_(-7)
        out_d.fill_(0.0)
        dade.dade_search(gi, Qd, w.k, w.nprobe, out_ids=out_i, out_dist2=out_d, use_graph=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out_i), ref_i)
        assert np.array_equal(to_np(out_d).view(np.uint32), ref_d.view(np.uint32))
        gpu_search(gi, Qd[:7].contiguous(), 5, 3, use_graph=False)   # eager work between replays


def test_all_lists_full_d_is_brute_force(small):
    """FDScanning over every list is brute-force KNN: the same ids, except where the FP64
    distances of the ids that differ tie with the K-th within the FP32 tolerance."""
    w = small["w"]
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"][:40], 10, w.nlist, mode="full_d")
    gt, gd = knn.brute_force(small["X"], small["Q"][:40], 10)
    np.testing.assert_allclose(g_d2, gd, rtol=1e-5)
    ex = exact_d2(small["X"], small["Q"][:40], g_ids)
    for qi in range(len(gt)):
        for i in set(g_ids[qi].tolist()) ^ set(gt[qi].tolist()):
            d = ex[qi][g_ids[qi] == i][0] if i in g_ids[qi] else gd[qi][gt[qi] == i][0]
            assert abs(d - gd[qi, -1]) <= 1e-5 * gd[qi, -1], (qi, i)


@pytest.mark.parametrize("nprobe", [100, 160])
def test_probe_selection_beyond_64_probes(small, nprobe):
    """160 lists and 100 or all 160 probes (the probe selection's threshold from a radix
    selection rather than the lane-minimum search): DADE results and DCO counts as the oracle's."""
    w = small["w"]
    X, Q = small["X"], small["Q"][:60]
    oi, _, _ = oracle_index(X, 160, w.seed, alpha=w.alpha)
    gi = dade.dade_import(artifacts(oi), small["Xd"])
    o = oracle_ivf(oi, Q, w.k, nprobe, w.delta_d)
    stats = torch.zeros((len(Q), 4), dtype=torch.int64, device="cuda")
    g_ids, g_d2 = gpu_search(gi, small["Qd"][:60].contiguous(), w.k, nprobe, delta_d=w.delta_d, stats=stats)
    compare(o, g_ids, g_d2, X, Q, w.k)
    same = o.logs["probe_gap"] > 1e-5   # no near tie in the probe order: the same candidates
    np.testing.assert_array_equal(to_np(stats)[same, 0], o.logs["dcos"][same].astype(np.int64))
    gi.close()


@pytest.mark.parametrize("store,rule", [("f32", "all"), ("bf16", "all"), ("bf16", "lazy")])
def test_exact_integer_inputs_match_bit_for_bit(store, rule):
    """Where FP32 is exact, nothing may be excused: every query's ids, distances (bit for bit),
    DCO count and dimensions read equal the oracle's, over schedules, round shapes, K and
    Delta_d -- including exact distance ties (duplicate rows) broken by id on the device."""
    _need_gpu()
    delta = 2.0 ** -10
    X, Q, oi = integer_index(store, delta)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda(), store=store)
    Qd = torch.from_numpy(Q).cuda()
    for K, npb, dd, sched, fill, growth in ((10, 3, 8, "per_rank", 32, 16), (10, 4, 8, "doubling", 32, 0),
                                            (1, 2, 8, "per_rank", 0, 0), (25, 5, 16, "doubling", 0, 2),
                                            (7, 16, 4, "doubling", 32, 0)):
        kw = dict(schedule=sched, fill_min=fill, growth=growth)
        o_ids, o_d2, logs = ivf.search(oi, Q, K, npb, dd, log=True, rerank=rule, **kw)
        stats = torch.zeros((len(Q), 4), dtype=torch.int64, device="cuda")
        g_ids, g_d2 = gpu_search(gi, Qd, K, npb, delta_d=dd, stats=stats, rerank_delta=delta, rerank_rule=rule, **kw)
        st = to_np(stats)
        assert np.array_equal(g_ids, o_ids), (K, npb, dd, sched)
        assert np.array_equal(g_d2.astype(np.float64), o_d2), (K, npb, dd, sched)
        np.testing.assert_array_equal(st[:, 0], logs["dcos"].astype(np.int64))
        np.testing.assert_array_equal(st[:, 1], logs["dims"].astype(np.int64))
        assert (g_d2[:15, 0] == 0).all()          # the queries that are rows find them at distance 0
    gi.close()


def test_uneven_k_and_nprobe(small):
    w, oi = small["w"], small["oi"]
    K, npb = workloads.uneven_batch(w.n_queries, 1, 40, (1, 10, 50, 100), seed=3)
    o = oracle_ivf(oi, small["Q"], K, np.minimum(npb, w.nlist), w.delta_d)
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"], 100, 40, delta_d=w.delta_d,
                             k_per_query=torch.from_numpy(K).cuda(),
                             nprobe_per_query=torch.from_numpy(npb).cuda())
    compare(o, g_ids, g_d2, small["X"], small["Q"], K)


def test_batch_invariance_bitwise(small):
    w = small["w"]
    ids_b, d2_b = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, delta_d=w.delta_d)
    for qi in (0, 17, 99):
        ids_1, d2_1 = gpu_search(small["gi"], small["Qd"][qi:qi + 1].contiguous(), w.k, w.nprobe,
                                 delta_d=w.delta_d)
        assert np.array_equal(ids_1[0], ids_b[qi])
        assert np.array_equal(d2_1[0].view(np.uint32), d2_b[qi].view(np.uint32))
    # a permuted batch gives the same per-query rows
    perm = np.random.default_rng(0).permutation(w.n_queries)
    ids_p, d2_p = gpu_search(small["gi"], small["Qd"][torch.from_numpy(perm).cuda()].contiguous(), w.k,
                             w.nprobe, delta_d=w.delta_d)
    assert np.array_equal(ids_p, ids_b[perm]) and np.array_equal(d2_p, d2_b[perm])


@pytest.mark.parametrize("dd", [5, 8, 64, 128])
def test_delta_d_variants(small, dd):
    """Delta_d not a multiple of 8 (per-dimension tests), several tests per chunk, none."""
    w, oi = small["w"], small["oi"]
    o = oracle_ivf(oi, small["Q"], w.k, w.nprobe, dd)
    g_ids, g_d2 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, delta_d=dd)
    compare(o, g_ids, g_d2, small["X"], small["Q"], w.k)


def test_k_larger_than_candidates_pads():
    _need_gpu()
    X, Q = workloads.make_mixture(300, 40, 4, 1.2, 6, seed=8)
    oi, _, _ = oracle_index(X, 32, 8, n_pairs=5000)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda())
    o = oracle_ivf(oi, Q, 128, 1, 8)
    g_ids, g_d2 = gpu_search(gi, torch.from_numpy(Q).cuda(), 128, 1, delta_d=8)
    compare(o, g_ids, g_d2, X, Q, 128)
    assert (g_ids == -1).any()   # one list holds fewer than 128 rows


def test_odd_dimension_and_nprobe_clamp():
    """D = 100 (padded to 128 inside), nprobe > nlist clamps to nlist, K = 1."""
    _need_gpu()
    X, Q = workloads.make_mixture(4000, 100, 8, 1.1, 30, seed=9)
    oi, _, _ = oracle_index(X, 16, 9, n_pairs=20000)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda())
    for K, npb, dd in ((1, 100, 24), (7, 3, 25)):
        o = oracle_ivf(oi, Q, K, npb, dd)
        g_ids, g_d2 = gpu_search(gi, torch.from_numpy(Q).cuda(), K, npb, delta_d=dd)
        compare(o, g_ids, g_d2, X, Q, K)


def test_empty_batch_is_a_noop(small):
    ids = torch.full((0, 10), 7, dtype=torch.int64, device="cuda")
    d2 = torch.zeros((0, 10), dtype=torch.float32, device="cuda")
    dade.dade_search(small["gi"], small["Qd"][:0], 10, 8, out_ids=ids, out_dist2=d2)
    torch.cuda.synchronize()


def test_gpu_build_rotate_calibrate_match_oracle(small):
    """Build stage (the library's own offline path) against the oracle on the same X."""
    w, X, oi = small["w"], small["X"], small["oi"]
    g = dade.dade_build_index(small["Xd"], w.nlist, init_rows=small["init"])
    art = dade.dade_export(g)
    # k-means: same seed rows, FP32 vs FP64 -- objectives agree to 1e-3
    lab_g = np.empty(w.n, np.int64)
    for l in range(w.nlist):
        lab_g[art["list_ids"][art["list_offsets"][l]:art["list_offsets"][l + 1]]] = l
    obj_g = ivf.objective(X, art["centroids"], lab_g)
    obj_o = ivf.objective(X, oi.centroids, ivf.assign(X, oi.centroids))
    assert abs(obj_g - obj_o) / obj_o < 1e-3
    # lists: ascending ids, each row's list is its nearest centroid (FP32 near ties excused)
    d2c = cdist(X.astype(np.float64), art["centroids"], "sqeuclidean")
    best = d2c.min(1)
    assert np.mean(d2c[np.arange(w.n), lab_g] <= best * (1 + 1e-5) + 1e-6) == 1.0
    dade.dade_rotate(g)
    art = dade.dade_export(g)
    np.testing.assert_allclose(art["lam"], oi.lam, rtol=1e-9, atol=1e-12 * oi.lam[0])
    W = art["W"]
    assert np.max(np.abs(W.T @ W - np.eye(w.dim))) < 1e-12
    gap = np.abs(np.diff(oi.lam)) / oi.lam[:-1]
    for kk in range(w.dim):
        ok_gap = (kk == 0 or gap[kk - 1] > 1e-6) and (kk == w.dim - 1 or gap[kk] > 1e-6)
        if ok_gap:
            assert abs(W[:, kk] @ oi.W[:, kk]) > 1 - 1e-8, kk
    np.testing.assert_allclose(art["mu"], oi.mu, rtol=1e-12, atol=1e-12)
    dade.dade_calibrate(g, w.alpha, pairs=small["pairs"])
    T = dade.dade_export(g)["T"]
    assert np.max(np.abs(T - oi.T)) < 1e-9
    # and the library's own index searches like the oracle's (recall within a hair)
    g_ids, _ = gpu_search(g, small["Qd"], w.k, w.nprobe, delta_d=w.delta_d)
    gt, _ = knn.brute_force(X, small["Q"], w.k)
    o_ids, _ = ivf.search(oi, small["Q"], w.k, w.nprobe, w.delta_d)
    assert abs(knn.recall(g_ids, gt, w.k).mean() - knn.recall(o_ids, gt, w.k).mean()) < 0.02
    g.close()


@pytest.mark.parametrize("store", ["bf16", "f16"])
def test_low_precision_store(small, store):
    """BF16/FP16 store + FP32 rerank: distances exact to FP32, recall close to the FP32 path,
    thresholds calibrated on stored coordinates close to the oracle's."""
    w, X, Q = small["w"], small["X"], small["Q"]
    ol, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha, store=store)
    gl = dade.dade_import(artifacts(ol), small["Xd"], store=store)
    g_ids, g_d2 = gpu_search(gl, small["Qd"], w.k, w.nprobe, delta_d=w.delta_d)
    ex = exact_d2(X, Q, g_ids)
    np.testing.assert_allclose(g_d2, ex, rtol=1e-5)
    o_ids, _ = ivf.search(ol, Q, w.k, w.nprobe, w.delta_d)
    f_ids, _ = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, delta_d=w.delta_d)
    gt, _ = knn.brute_force(X, Q, w.k)
    r_low, r_f32, r_or = (knn.recall(a, gt, w.k).mean() for a in (g_ids, f_ids, o_ids))
    assert abs(r_low - r_or) < 0.02 and r_low > r_f32 - 0.02
    # the library's own calibration on its stored coordinates
    dade.dade_calibrate(gl, w.alpha, pairs=small["pairs"])
    T = dade.dade_export(gl)["T"]
    assert np.max(np.abs(T - ol.T)) < 2e-3
    gl.close()


def _identity_rotation_case(store, delta, rule, dim, searches):
    """An index with W = I and mu = 0 (the library's stored coordinates are then exactly the
    oracle's rounded X), searched on the GPU and by the oracle; ids compared as everywhere."""
    from oracle import estimator, lowp
    X, Q = workloads.make_mixture(6000, dim, 12, 1.2, 60, seed=13)
    init = workloads.kmeans_init_rows(len(X), 24, 13)
    pairs = workloads.calibration_pairs(len(X), 30000, 13)
    lam = np.sort(np.var(X.astype(np.float64), axis=0))[::-1].copy()
    Ys = lowp.store(X.astype(np.float64), store)
    eps, T, _ = estimator.calibrate(X, np.eye(dim), lam, pairs, 0.1, stored=Ys)
    C = ivf.kmeans(X, init, 10)
    off, ids = ivf.build_lists(ivf.assign(X, C), 24)
    oi = ivf.Index(np.zeros(dim), np.eye(dim), lam, eps, C, off, ids, Ys,
                   Y_exact=X.astype(np.float64), delta=delta, T=T)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda(), store=store)
    for K, npb, sched in searches:
        o = oracle_ivf(oi, Q, K, npb, 16, schedule=sched, rerank=rule)
        g_ids, g_d2 = gpu_search(gi, torch.from_numpy(Q).cuda(), K, npb, delta_d=16, schedule=sched,
                                 rerank_delta=delta, rerank_rule=rule)
        compare(o, g_ids, g_d2, X, Q, K)
    gi.close()


@pytest.mark.parametrize("rule", ["all", "lazy"])
@pytest.mark.parametrize("store,delta", [("bf16", 0.02), ("f16", 0.002), ("bf16", 0.0)])
def test_low_precision_rerank_rule_parity(store, delta, rule):
    """With W = I and mu = 0 the library's stored coordinates are exactly the oracle's rounded
    X, so the rerank rule (gate, K smallest, bound from the K-th exact) is compared ID for ID."""
    _need_gpu()
    _identity_rotation_case(store, delta, rule, 64, ((10, 4, "per_rank"), (25, 6, "doubling"), (1, 3, "per_rank")))


@pytest.mark.parametrize("rule", ["all", "lazy"])
def test_low_precision_odd_dimension(rule):
    """D = 100 with a BF16 store (rows padded to 128: the last block is partly padding) over the
    three schedules; the heap-filling rounds read whole rows, whose query chunks are staged per
    step of blocks, so their clamped loads and the +0 addends past D are exercised."""
    _need_gpu()
    _identity_rotation_case("bf16", 0.02, rule, 100, ((10, 4, "whole"), (25, 6, "doubling"), (1, 3, "per_rank")))


def test_data_oblivious_rotation_matches_oracle():
    """The data-oblivious comparison (a seeded Haar rotation in place of the data-aware W, Figure 1)
    through the same boundary: imported, calibrated on the GPU (T_d as the oracle's), and searched
    as the oracle searches the same index."""
    _need_gpu()
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w)
    rot = workloads.oblivious_rotation(w.dim, w.seed)
    init = workloads.kmeans_init_rows(len(X), w.nlist, w.seed)
    pairs = workloads.calibration_pairs(len(X), 100_000, w.seed)
    oi = ivf.build(X, w.nlist, init, pairs, p_s=w.alpha, iters=10, rotation=rot)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    art = artifacts(oi)
    art["T"] = None
    gi = dade.dade_import(art, Xd)
    dade.dade_calibrate(gi, w.alpha, pairs=pairs)
    assert np.max(np.abs(dade.dade_export(gi)["T"] - oi.T)) < 1e-9
    o = oracle_ivf(oi, Q, w.k, w.nprobe, w.delta_d, schedule="doubling")
    logs = o.logs
    stats = torch.zeros((w.n_queries, 4), dtype=torch.int64, device="cuda")
    g_ids, g_d2 = gpu_search(gi, Qd, w.k, w.nprobe, delta_d=w.delta_d, schedule="doubling", stats=stats)
    compare(o, g_ids, g_d2, X, Q, w.k)
    st = to_np(stats)
    np.testing.assert_array_equal(st[:, 0], logs["dcos"].astype(np.int64))
    rel = np.abs(st[:, 1] - logs["dims"]) / logs["dims"]
    assert np.median(rel) == 0.0 and rel.max() < 0.02
    gi.close()


@pytest.mark.parametrize("dd", [1, 4, 16])
def test_linear_scan_one_list(dd):
    """One list holding every row (the linear-scan study): growth-capped rounds inside the list
    and DADE at small Delta_d (per-dimension tests for 1 and 4), against the oracle."""
    _need_gpu()
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n=4000, n_queries=24)
    oi, _, _ = oracle_index(X, 1, w.seed, n_pairs=20000, alpha=w.alpha)
    gi = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda())
    Qd = torch.from_numpy(Q).cuda()
    sched = dict(schedule="doubling", fill_min=32, growth=16)
    o = oracle_ivf(oi, Q, w.k, 1, dd, **sched)
    logs = o.logs
    stats = torch.zeros((len(Q), 4), dtype=torch.int64, device="cuda")
    g_ids, g_d2 = gpu_search(gi, Qd, w.k, 1, delta_d=dd, stats=stats, **sched)
    compare(o, g_ids, g_d2, X, Q, w.k)
    st = to_np(stats)
    np.testing.assert_array_equal(st[:, 0], logs["dcos"].astype(np.int64))
    rel = np.abs(st[:, 1] - logs["dims"]) / logs["dims"]
    assert np.median(rel) == 0.0 and rel.max() < 0.02
    gi.close()


def test_stage_times_of_a_timed_search(small):
    """A timed search (kernels launched one by one, events around each) gives the same rows as
    the untimed one; its report counts every round's DCO kernel and the kernels fit in the stage."""
    w = small["w"]
    kw = dict(delta_d=w.delta_d, schedule="doubling", fill_min=32, growth=0)
    ids0, d0 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, **kw)
    ids1, d1 = gpu_search(small["gi"], small["Qd"], w.k, w.nprobe, record_times=True, **kw)
    assert np.array_equal(ids0, ids1) and np.array_equal(d0.view(np.uint32), d1.view(np.uint32))
    t = dade.dade_stage_times(small["gi"])
    rounds = 2 + int(np.ceil(np.log2(w.nprobe)))   # the first round, then ranks 1, 2, 4, ... nprobe
    assert t["round_launches"] == rounds
    assert t["round_kernel_ms"] > 0 and t["merge_kernel_ms"] > 0 and t["plan_ms"] > 0
    assert t["round_kernel_ms"] + t["merge_kernel_ms"] + t["plan_ms"] <= t["scan_ms"] * 1.01
