"""The benchmark's host logic on the CPU: its refusal of more than one GPU, and the graph study's
control flow (two builds, the sweep, the visited-table bound on expansions, the headline pick)
run against stand-ins for the library and torch that return fixed values."""
import os
import subprocess
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class _Arr:
    """A host array dressed as the few tensor methods the study calls."""

    def __init__(self, a):
        self.a = np.asarray(a)

    def cpu(self):
        return self

    def numpy(self):
        return self.a

    def cuda(self):
        return self

    @property
    def shape(self):
        return self.a.shape

    @property
    def device(self):
        return "cuda"


class _Event:
    def __init__(self, **kw):
        pass

    def record(self):
        pass

    def elapsed_time(self, other):
        return 1.0


def test_graph_study_control_flow(monkeypatch):
    width = [0]
    calls = []

    def build(ix, degree, reverse, nprobe, candidates):
        width[0] = degree + reverse
        calls.append((degree, reverse, nprobe, candidates))

    def search(ix, Qd, k, ef, stats=None, n_entry=4, delta_d=32, mode="dade", max_iters=0):
        # the library's bounds: k <= ef <= 64, 2 n_entry + max_iters x width <= 4096
        assert 1 <= k <= ef <= 64 and 1 <= max_iters <= 2 * ef
        assert 2 * n_entry + max_iters * width[0] <= 4096
        nq = Qd.shape[0]
        if stats is not None:
            stats.a[:] = [100, 1000, 10, 100]
        return _Arr(np.tile(np.arange(k), (nq, 1))), None

    class _Index:
        def close(self):
            pass

    dade = types.SimpleNamespace(dade_build_index=lambda *a, **k: _Index(), dade_rotate=lambda ix: None,
                                 dade_calibrate=lambda *a, **k: None, dade_graph_build=build,
                                 dade_graph_search=search)
    torch = types.SimpleNamespace(from_numpy=_Arr, int64=None,
                                  zeros=lambda shape, dtype=None, device=None: _Arr(np.zeros(shape, np.int64)),
                                  cuda=types.SimpleNamespace(Event=_Event, synchronize=lambda: None))
    monkeypatch.setattr(bench, "ground_truth", lambda torch_, Xd, Qd, k: np.tile(np.arange(k), (Qd.shape[0], 1)))
    out = bench.graph_study(dade, torch, 0.95, 2)
    assert sorted(out["builds"]) == sorted(bench.GRAPH_BUILDS)
    assert len(calls) == len(bench.GRAPH_BUILDS)
    # the selected build probes every list of the index
    sel = out["builds"]["hnsw_select"]
    assert sel["nprobe_build"] == out["nlist"] and sel["candidates"] > sel["degree"]
    for b in out["builds"].values():
        for mode in ("dade", "full_d"):
            assert len(b["sweep"][mode]) == len(bench.GRAPH_ENTRY) * len(bench.GRAPH_EF)
    for mode in ("dade", "full_d"):
        assert out[mode]["build"] in out["builds"] and out[mode]["recall@10"] == 1.0
    assert out["speedup_vs_full_d"] > 0
