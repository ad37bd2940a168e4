"""The serving loop (dade_serve) on the GPU: requests admitted by a device budget and batched as
they arrive give, for every query, exactly the rows dade_search gives for its request alone
(bitwise), and those rows match the oracle; budget waits, rejections and latencies are
reported as specified."""
import numpy as np
import pytest

from oracle import ivf
from paper_2411_17229_amd import dade, workloads
from gpu_helpers import artifacts, compare, oracle_ivf, oracle_index, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KW = dict(delta_d=32, schedule="doubling", fill_min=32, growth=0)
K_MAX, NP_MAX = 50, 64


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n_queries=600)
    oi, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha)
    Xd = torch.from_numpy(X).cuda()
    gi = dade.dade_import(artifacts(oi), Xd)
    return dict(w=w, X=X, Q=Q, Qd=torch.from_numpy(Q).cuda(), oi=oi, gi=gi)


def request_mix(n_req, total_cap, seed, rate=1e9):
    """Seeded requests (sizes log-uniform in 1..256 as the serving workload's, cut to fit
    `total_cap` queries), K in {1, 10, 50}, nprobe in {4, 8, 64}."""
    arr, sizes, ks, nps = workloads.requests(n_req, rate, ks=(1, 10, 50), nprobes=(4, 8, 64), seed=seed)
    sizes = np.minimum(sizes, 48).astype(np.int32)
    keep = np.cumsum(sizes) <= total_cap
    return arr[keep], sizes[keep], ks[keep], nps[keep]


def alone_rows(env, a, b, k, nprobe):
    ids, d2 = dade.dade_search(env["gi"], env["Qd"][a:b].contiguous(), k, nprobe, **KW)
    torch.cuda.synchronize()
    return to_np(ids), to_np(d2)


def check_against_alone(env, sizes, ks, nps, ids, d2, skip=()):
    starts = np.concatenate([[0], np.cumsum(sizes)])
    for r in range(len(sizes)):
        a, b, k = int(starts[r]), int(starts[r + 1]), int(ks[r])
        if r in skip:
            continue
        i1, d1 = alone_rows(env, a, b, k, int(nps[r]))
        assert np.array_equal(ids[a:b, :k], i1), r
        assert np.array_equal(d2[a:b, :k].view(np.uint32), d1.view(np.uint32)), r
        assert np.all(ids[a:b, k:] == -1) and np.all(np.isinf(d2[a:b, k:])), r


def workspace_bytes(env):
    """The search workspace the loop holds for launches of 48 queries (48 one-query requests:
    the loop sizes it for min(max_batch, all queries))."""
    one = np.ones(48, np.int32)
    _, _, _, st = dade.dade_serve(env["gi"], np.zeros(48), one, one, one, env["Q"][:48], K_MAX, NP_MAX, max_batch=48,
                                  **KW)
    return st["workspace_bytes"]


def slot_bytes(dim):
    return dim * 4 + 8 + K_MAX * 12


@pytest.mark.parametrize("pinned", [False, True])
def test_burst_batches_split_and_wait(env, pinned):
    """Every request arrives at once; launches of at most 48 queries split requests across
    launches, and a ring of 100 slots makes later requests wait for earlier ones.  Queries in
    pageable memory are staged; pinned ones are copied from where they are."""
    arr, sizes, ks, nps = request_mix(80, 600, seed=1)
    arr = np.zeros_like(arr)
    Qs = env["Q"][: int(sizes.sum())]
    if pinned:
        Qs = torch.from_numpy(Qs).pin_memory()
    budget = workspace_bytes(env) + 100 * slot_bytes(env["w"].dim)
    ids, d2, lat, st = dade.dade_serve(env["gi"], arr, sizes, ks, nps, Qs, K_MAX, NP_MAX, budget_bytes=budget,
                                       max_batch=48, max_inflight=2, **KW)
    assert st["served_requests"] == len(sizes) and st["rejected_requests"] == 0
    assert st["served_queries"] == sizes.sum()
    assert st["ring_slots"] == 100 and st["peak_slots"] <= 100
    assert st["waited_requests"] > 0
    assert st["launches"] >= int(np.ceil(sizes.sum() / 48))
    assert np.all(lat >= 0) and st["wall_s"] >= lat.max() - 1e-9
    check_against_alone(env, sizes, ks, nps, ids, d2)


def test_poisson_arrivals_match_alone_and_oracle(env):
    """Requests arriving over ~50 ms: per-request latencies, results equal to each request alone,
    and to the oracle (up to near ties) on every query."""
    arr, sizes, ks, nps = request_mix(200, 600, seed=2, rate=400.0)
    total = int(sizes.sum())
    Qs = env["Q"][:total]
    ids, d2, lat, st = dade.dade_serve(env["gi"], arr, sizes, ks, nps, Qs, K_MAX, NP_MAX, max_batch=64, **KW)
    assert st["served_requests"] == len(sizes) and np.all(lat >= 0)
    assert st["wall_s"] >= arr[-1]
    check_against_alone(env, sizes, ks, nps, ids, d2)
    K = np.repeat(ks, sizes)
    npb = np.repeat(nps, sizes)
    o = oracle_ivf(env["oi"], Qs, K, np.minimum(npb, env["w"].nlist), 32, schedule="doubling",
                   fill_min=32, growth=0)
    compare(o, ids, d2, env["X"], Qs, K)


@pytest.mark.parametrize("pinned", [False, True])
def test_requests_larger_than_the_ring_are_rejected(env, pinned):
    """A ring of 20 slots: requests of more than 20 queries are rejected (rows (-1, +inf),
    latency -1); the others are served as alone.  With pinned queries a launch's rows are not
    one run of Q when a rejected request sits between its requests."""
    arr, sizes, ks, nps = request_mix(60, 600, seed=3)
    assert (sizes > 20).any() and (sizes <= 20).any()
    Qs = env["Q"][: int(sizes.sum())]
    if pinned:
        Qs = torch.from_numpy(Qs).pin_memory()
    budget = workspace_bytes(env) + 20 * slot_bytes(env["w"].dim)
    ids, d2, lat, st = dade.dade_serve(env["gi"], arr, sizes, ks, nps, Qs, K_MAX, NP_MAX, budget_bytes=budget,
                                       max_batch=16, **KW)
    big = np.flatnonzero(sizes > 20)
    assert st["rejected_requests"] == len(big) and st["served_requests"] == len(sizes) - len(big)
    assert np.all(lat[big] == -1.0) and np.all(lat[sizes <= 20] >= 0)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    for r in big:
        assert np.all(ids[starts[r]:starts[r + 1]] == -1) and np.all(np.isinf(d2[starts[r]:starts[r + 1]]))
    check_against_alone(env, sizes, ks, nps, ids, d2, skip=set(big.tolist()))


def test_argument_errors(env):
    gi, Q = env["gi"], env["Q"]
    with pytest.raises(dade.DadeError):   # K above k_max
        dade.dade_serve(gi, [0.0], [1], [K_MAX + 1], [4], Q[:1], K_MAX, NP_MAX, **KW)
    with pytest.raises(dade.DadeError):   # arrivals out of order
        dade.dade_serve(gi, [0.1, 0.0], [1, 1], [1, 1], [4, 4], Q[:2], K_MAX, NP_MAX, **KW)
    with pytest.raises(dade.DadeError):   # a budget below the search workspace
        dade.dade_serve(gi, [0.0], [1], [1], [4], Q[:1], K_MAX, NP_MAX, budget_bytes=1024, **KW)
    ids, d2, lat, st = dade.dade_serve(gi, [], [], [], [], Q[:0], K_MAX, NP_MAX, **KW)
    assert ids.shape == (0, K_MAX) and st["served_requests"] == 0
