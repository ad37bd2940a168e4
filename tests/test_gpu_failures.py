"""Error paths forced from the host: device allocations refused through the library's
DADE_FAIL_ALLOC_AFTER hook (no kernel sees a missing buffer: every call checks its allocations
before launching).  Each refused call returns DADE_ENOMEM, and the same call succeeds once
allocations are allowed again, with the index giving the results it gave before."""
import numpy as np
import pytest

from paper_2411_17229_amd import dade, workloads
from gpu_helpers import to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HOOK = "DADE_FAIL_ALLOC_AFTER"
KW = dict(delta_d=32, schedule="doubling", fill_min=32, growth=0)


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    w = workloads.WORKLOADS["small-20k-d128"]
    X, Q = workloads.make(w, n_queries=300)
    return w, torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()


def refused(monkeypatch, n_ok, fn):
    monkeypatch.setenv(HOOK, str(n_ok))
    with pytest.raises(dade.DadeError) as e:
        fn()
    monkeypatch.delenv(HOOK)
    assert e.value.code == dade.DADE_ENOMEM and HOOK in str(e.value)


def test_build_rotate_search_and_serve_recover_from_refused_allocations(data, monkeypatch):
    w, Xd, Qd = data
    init = workloads.kmeans_init_rows(w.n, w.nlist, w.seed)
    for n_ok in (0, 1, 3, 6):   # the build fails at different allocations and frees what it took
        refused(monkeypatch, n_ok, lambda: dade.dade_build_index(Xd, w.nlist, init_rows=init))
    gi = dade.dade_build_index(Xd, w.nlist, init_rows=init)
    refused(monkeypatch, 0, lambda: dade.dade_rotate(gi))
    dade.dade_rotate(gi)
    dade.dade_calibrate(gi, w.alpha, pairs=workloads.calibration_pairs(w.n, 20_000, w.seed))
    ids10, d10 = dade.dade_search(gi, Qd[:10].contiguous(), w.k, w.nprobe, **KW)
    ids10, d10 = to_np(ids10), to_np(d10)
    # a larger batch needs a larger workspace: refused, then served, and the first 10 rows agree
    refused(monkeypatch, 0, lambda: dade.dade_search(gi, Qd, w.k, w.nprobe, **KW))
    ids, d2 = dade.dade_search(gi, Qd, w.k, w.nprobe, **KW)
    torch.cuda.synchronize()
    dade.dade_check(gi)
    assert np.array_equal(to_np(ids)[:10], ids10) and np.array_equal(to_np(d2)[:10].view(np.uint32),
                                                                      d10.view(np.uint32))
    # the serving loop's ring allocation refused, then the same requests served
    Qh = Qd.cpu().numpy()
    args = (np.zeros(3), np.array([4, 2, 4], np.int32), np.full(3, w.k, np.int32), np.full(3, w.nprobe, np.int32),
            Qh[:10], w.k, w.nprobe)
    refused(monkeypatch, 0, lambda: dade.dade_serve(gi, *args, **KW))
    s_ids, _, lat, st = dade.dade_serve(gi, *args, **KW)
    assert st["served_requests"] == 3 and np.array_equal(s_ids, ids10)
    gi.close()
