"""The allocation-free search entry point (dade_search_noalloc) against dade_search: the same rows
bit for bit, on two calls in a row (the second smaller), across slices of its fixed scratch,
with every device allocation of the library refused, and its errors."""
import os

import numpy as np
import pytest

from gpu_helpers import artifacts, oracle_index, to_np
from paper_2411_17229_amd import dade, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n_queries=400)
    oi, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha)
    f32 = dade.dade_import(artifacts(oi), torch.from_numpy(X).cuda())
    ol, _, _ = oracle_index(X, w.nlist, w.seed, alpha=w.alpha, store="bf16")
    b16 = dade.dade_import(artifacts(ol), torch.from_numpy(X).cuda(), store="bf16")
    yield dict(w=w, Qd=torch.from_numpy(Q).cuda(), f32=f32, bf16=b16)
    f32.close()
    b16.close()


def _both(ix, Qd, k, nprobe, **kw):
    nq = Qd.shape[0]
    ref_i, ref_d = dade.dade_search(ix, Qd, k, nprobe, use_graph=False, **kw)
    out_i = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    out_d = torch.zeros((nq, k), dtype=torch.float32, device="cuda")
    rec = {}
    dade.dade_search_noalloc(ix, Qd, k, nprobe, out_i, out_d, record=rec, **kw)
    torch.cuda.synchronize()
    dade.dade_check(ix)
    return to_np(ref_i), to_np(ref_d), to_np(out_i), to_np(out_d), rec


@pytest.mark.parametrize("store,kw", [("f32", dict(delta_d=32)),
                                      ("f32", dict(delta_d=16, schedule="doubling", fill_min=32, growth=0)),
                                      ("bf16", dict(delta_d=32, schedule="doubling", growth=0)),
                                      ("bf16", dict(delta_d=32, rerank_rule="lazy"))])
def test_noalloc_matches_search_on_two_calls(env, store, kw):
    ix = env[store]
    for nq, k, nprobe in ((400, 10, 8), (37, 25, 5)):   # the second call smaller
        Qd = env["Qd"][:nq].contiguous()
        ri, rd, gi, gd, rec = _both(ix, Qd, k, nprobe, **kw)
        assert np.array_equal(gi, ri) and np.array_equal(gd.view(np.uint32), rd.view(np.uint32)), (nq, k)
        assert rec["passes"] == 1 and rec["graph"] == 0 and rec["k"] == k


def test_noalloc_with_every_device_allocation_refused(env):
    """With the library's device allocations refused, dade_search_noalloc still runs (it allocates
    nothing) while a search that must grow its workspace fails with DADE_ENOMEM."""
    ix, Qd = env["f32"], env["Qd"]
    ri, rd = dade.dade_search(ix, Qd, 10, 8, use_graph=False)
    torch.cuda.synchronize()
    out_i = torch.empty((len(Qd), 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((len(Qd), 10), dtype=torch.float32, device="cuda")
    grown_i = torch.empty((len(Qd), 128), dtype=torch.int64, device="cuda")
    grown_d = torch.empty((len(Qd), 128), dtype=torch.float32, device="cuda")
    os.environ["DADE_FAIL_ALLOC_AFTER"] = "0"
    try:
        dade.dade_search_noalloc(ix, Qd, 10, 8, out_i, out_d)
        torch.cuda.synchronize()
        with pytest.raises(dade.DadeError) as e:
            dade.dade_search(ix, Qd, 128, 64, out_ids=grown_i, out_dist2=grown_d)   # needs a larger workspace
        assert e.value.code == dade.DADE_ENOMEM
    finally:
        del os.environ["DADE_FAIL_ALLOC_AFTER"]
    assert np.array_equal(to_np(out_i), to_np(ri)) and np.array_equal(to_np(out_d), to_np(rd))


def test_noalloc_runs_large_batches_in_slices(env):
    """A batch larger than the scratch holds runs in slices; rows equal dade_search's."""
    ix = env["f32"]
    reps = 60
    Qd = env["Qd"].repeat(reps, 1).contiguous()   # 24,000 queries
    ri, rd, gi, gd, rec = _both(ix, Qd, 100, 64, delta_d=32)
    assert rec["passes"] > 1, rec
    assert np.array_equal(gi, ri) and np.array_equal(gd.view(np.uint32), rd.view(np.uint32))


def test_noalloc_rejects_a_query_larger_than_the_scratch():
    """One list of 3M rows, per-rank rounds growing by 2x: one query's workspace (its queued keys
    and work items over about 18 rounds) exceeds the 64 MiB scratch; the call is refused with a
    message naming the scratch, before any device work; dade_search runs it."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    n, D = 3_000_000, 8
    X = np.random.default_rng(5).standard_normal((n, D)).astype(np.float32)
    art = dict(W=np.eye(D), mu=np.zeros(D), lam=np.ones(D), centroids=np.zeros((1, D)),
               list_offsets=np.array([0, n]), list_ids=np.arange(n), T=np.linspace(0.2, 1.0, D))
    ix = dade.dade_import(art, torch.from_numpy(X).cuda())
    Qd = torch.from_numpy(X[:2] + 0.5).cuda()
    out_i = torch.empty((2, 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((2, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(dade.DadeError, match="scratch") as e:
        dade.dade_search_noalloc(ix, Qd, 10, 1, out_i, out_d, delta_d=4, growth=1)
    assert e.value.code == dade.DADE_EINVAL
    ids, _ = dade.dade_search(ix, Qd, 10, 1, delta_d=4, growth=1)
    torch.cuda.synchronize()
    assert (to_np(ids) >= 0).all()
    ix.close()


def test_noalloc_argument_errors(env):
    ix, Qd = env["f32"], env["Qd"]
    out_i = torch.empty((len(Qd), 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((len(Qd), 10), dtype=torch.float32, device="cuda")
    o = dade._search_opts()
    o.record_times = 1
    rc = dade.lib().dade_search_noalloc(ix.handle, dade._dev(Qd, torch.float32, "Q"), len(Qd), 10, 8, None, None,
                                        dade.ctypes.byref(o), dade._dev(out_i, torch.int64, "o"),
                                        dade._dev(out_d, torch.float32, "d"), dade._stream(None))
    assert rc == dade.DADE_EINVAL and "record_times" in dade.dade_last_error()
    with pytest.raises(dade.DadeError):
        dade.dade_search_noalloc(ix, Qd, 0, 8, out_i[:, :0], out_d[:, :0])
    with pytest.raises(ValueError):   # outputs of the wrong shape never reach the device
        dade.dade_search_noalloc(ix, Qd, 10, 8, out_i[:5], out_d[:5])
