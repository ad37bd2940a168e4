"""Python binding of the C ABI in include/dade.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device buffers are torch
tensors on the current HIP device (torch is used for memory and streams only); the stream
is ``torch.cuda.current_stream()`` unless one is passed.  The library must have been built
(``paper_2411_17229_amd.build.build()``); importing this module does not load it, the first
call does, and it raises if ``libdade.so`` is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdade.so")

DADE_OK, DADE_EINVAL, DADE_ESTATE, DADE_ENOMEM, DADE_EDEVICE = 0, -1, -2, -3, -4
DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
MODES = {"dade": 0, "full_d": 1}
SCHEDULES = {"per_rank": 0, "doubling": 1, "whole": 2}
RERANK_RULES = {"all": 0, "lazy": 1}
STATE_BUILT, STATE_ROTATED, STATE_CALIBRATED = 1, 2, 3
EXPORTED = ("dade_build_index", "dade_rotate", "dade_calibrate", "dade_search", "dade_search_noalloc",
            "dade_check", "dade_index_info",
            "dade_export", "dade_import", "dade_stage_times", "dade_serve", "dade_autotune", "dade_graph_build",
            "dade_graph_search", "dade_graph_export", "dade_destroy", "dade_last_error")
TUNE_MAX = 24


class DadeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("kmeans_iters", ctypes.c_int32), ("store_dtype", ctypes.c_int32),
                ("init_rows", ctypes.POINTER(ctypes.c_int64)), ("seed", ctypes.c_uint64),
                ("hbm_budget_bytes", ctypes.c_int64)]


class SearchRecord(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in ("delta_d", "mode", "schedule", "fill_min", "growth",
                                                      "rerank_rule")] + \
               [("rerank_delta", ctypes.c_float)] + \
               [(name, ctypes.c_int32) for name in ("k", "nprobe_requested", "nprobe", "nprobe_clamped", "rounds",
                                                      "passes", "graph")]


class SearchOpts(ctypes.Structure):
    _fields_ = [("delta_d", ctypes.c_int32), ("mode", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("rerank_delta", ctypes.c_float), ("stats", ctypes.c_void_p),
                ("record_times", ctypes.c_int32), ("fill_min", ctypes.c_int32), ("growth", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("scan_blocks_per_cu", ctypes.c_int32),
                ("rerank_rule", ctypes.c_int32), ("record", ctypes.POINTER(SearchRecord)),
                ("query_record", ctypes.c_void_p)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("nprobe_max", ctypes.c_int32), ("search", SearchOpts)]


class ServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("served_requests", ctypes.c_int64),
                ("rejected_requests", ctypes.c_int64), ("served_queries", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("ring_slots", ctypes.c_int64), ("peak_slots", ctypes.c_int64),
                ("waited_requests", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("stage_s", ctypes.c_double), ("launch_s", ctypes.c_double), ("retire_s", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("delta_d", ctypes.c_int32), ("schedule", ctypes.c_int32), ("fill_min", ctypes.c_int32),
                ("growth", ctypes.c_int32), ("scan_blocks_per_cu", ctypes.c_int32), ("ms", ctypes.c_float),
                ("agreement", ctypes.c_float)]


class Times(ctypes.Structure):
    _fields_ = [("query_gemm_ms", ctypes.c_float), ("select_ms", ctypes.c_float), ("scan_ms", ctypes.c_float),
                ("round_kernel_ms", ctypes.c_float), ("merge_kernel_ms", ctypes.c_float),
                ("plan_ms", ctypes.c_float), ("round_launches", ctypes.c_int32)]


class Artifacts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("nlist", ctypes.c_int32),
                ("store_dtype", ctypes.c_int32), ("state", ctypes.c_int32),
                ("W", ctypes.c_void_p), ("mu", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("delta", ctypes.c_double), ("centroids", ctypes.c_void_p),
                ("list_offsets", ctypes.c_void_p), ("list_ids", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libdade.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_17229_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.dade_build_index.argtypes = [vp, i64, i32, i32, ctypes.POINTER(BuildOpts), vp, pp]
        L.dade_rotate.argtypes = [vp, vp]
        L.dade_calibrate.argtypes = [vp, ctypes.c_double, vp, i64, u64, vp]
        L.dade_search.argtypes = [vp, vp, i64, i32, i32, vp, vp, ctypes.POINTER(SearchOpts), vp, vp, vp]
        L.dade_search_noalloc.argtypes = L.dade_search.argtypes
        L.dade_check.argtypes = [vp, vp]
        L.dade_index_info.argtypes = [vp] + [ctypes.POINTER(t) for t in (i64, i32, i32, i32, i32)]
        L.dade_export.argtypes = [vp, ctypes.POINTER(Artifacts)]
        L.dade_import.argtypes = [ctypes.POINTER(Artifacts), vp, ctypes.POINTER(BuildOpts), vp, pp]
        L.dade_stage_times.argtypes = [vp, ctypes.POINTER(Times)]
        L.dade_serve.argtypes = [vp, i64, vp, vp, vp, vp, vp, ctypes.POINTER(ServeOpts), vp, vp, vp,
                                 ctypes.POINTER(ServeStats), vp]
        L.dade_graph_build.argtypes = [vp, i32, i32, i32, i32, vp]
        L.dade_graph_search.argtypes = [vp, vp, i64, i32, i32, i32, i32, ctypes.POINTER(SearchOpts), vp, vp, vp]
        L.dade_graph_export.argtypes = [vp, ctypes.POINTER(i32), vp, vp]
        L.dade_autotune.argtypes = [vp, vp, i64, i32, i32, vp, vp, ctypes.c_float, i32, ctypes.POINTER(SearchOpts),
                                    ctypes.POINTER(TuneResult), ctypes.POINTER(i32), vp]
        L.dade_destroy.argtypes = [vp]
        L.dade_destroy.restype = None
        L.dade_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("dade_destroy", "dade_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != DADE_OK:
        raise DadeError(rc, lib().dade_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _shape(t, shape, name):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")


def _search_args(ix, Q, k, out_ids, out_dist2, k_per_query, nprobe_per_query, stats, query_record):
    """Shape checks of a search's tensors (the library reads and writes exactly these extents)."""
    nq = Q.shape[0]
    _shape(Q, (nq, ix.dim), "Q")
    _shape(out_ids, (nq, k), "out_ids")
    _shape(out_dist2, (nq, k), "out_dist2")
    for t, shape, name in ((k_per_query, (nq,), "k_per_query"), (nprobe_per_query, (nq,), "nprobe_per_query"),
                           (stats, (nq, 4), "stats"), (query_record, (nq, 3), "query_record")):
        if t is not None:
            _shape(t, shape, name)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


class Index:
    """Owns one dade_index handle."""

    def __init__(self, handle):
        self.handle = handle
        self._dim = None

    @property
    def dim(self):
        if self._dim is None:
            self._dim = dade_index_info(self)["dim"]
        return self._dim

    def info(self):
        return dade_index_info(self)

    def close(self):
        if self.handle:
            lib().dade_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _build_opts(store="f32", kmeans_iters=10, init_rows=None, seed=0, hbm_budget_bytes=0):
    o = BuildOpts()
    o.kmeans_iters = kmeans_iters
    o.store_dtype = DTYPES[store]
    keep = None
    if init_rows is not None:
        keep = np.ascontiguousarray(init_rows, dtype=np.int64)
        o.init_rows = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    o.seed = seed
    o.hbm_budget_bytes = hbm_budget_bytes
    return o, keep


def dade_build_index(X, nlist, store="f32", kmeans_iters=10, init_rows=None, seed=0,
                     hbm_budget_bytes=0, stream=None) -> Index:
    import torch
    p = _dev(X, torch.float32, "X")
    o, keep = _build_opts(store, kmeans_iters, init_rows, seed, hbm_budget_bytes)
    h = ctypes.c_void_p()
    _check(lib().dade_build_index(p, X.shape[0], X.shape[1], nlist, ctypes.byref(o), _stream(stream),
                                  ctypes.byref(h)))
    return Index(h)


def dade_rotate(ix: Index, stream=None):
    _check(lib().dade_rotate(ix.handle, _stream(stream)))


def dade_calibrate(ix: Index, alpha=0.1, pairs=None, n_pairs=100_000, seed=0, stream=None):
    if pairs is not None:
        pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
        n_pairs = pairs.shape[0]
        ptr = ctypes.c_void_p(pairs.ctypes.data)
    else:
        ptr = None
    _check(lib().dade_calibrate(ix.handle, float(alpha), ptr, n_pairs, seed, _stream(stream)))


def dade_search(ix: Index, Q, k, nprobe, k_per_query=None, nprobe_per_query=None, delta_d=0,
                mode="dade", schedule="per_rank", rerank_delta=-1.0, stats=None, record_times=False,
                out_ids=None, out_dist2=None, stream=None, fill_min=32, growth=16, use_graph=True,
                scan_blocks_per_cu=0, rerank_rule="all", record=None, query_record=None):
    """Returns (ids [nq, k] int64, dist2 [nq, k] float32) device tensors (asynchronous).

    ``record``: a dict filled with what the call ran with (dade_search_record's fields, the rerank
    rule and schedule by name); ``query_record``: a device int32 [nq, 3] tensor (K, nprobe used,
    rounds per query)."""
    import torch
    qp = _dev(Q, torch.float32, "Q")
    nq = Q.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
    if out_dist2 is None:
        out_dist2 = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    _search_args(ix, Q, k, out_ids, out_dist2, k_per_query, nprobe_per_query, stats, query_record)
    o = _search_opts(delta_d, mode, schedule, rerank_delta, fill_min, growth, use_graph, scan_blocks_per_cu,
                     rerank_rule)
    o.stats = None if stats is None else _dev(stats, torch.int64, "stats").value
    o.record_times = int(bool(record_times))
    o.query_record = None if query_record is None else _dev(query_record, torch.int32, "query_record").value
    rec = SearchRecord()
    if record is not None:
        o.record = ctypes.pointer(rec)
    kp = None if k_per_query is None else _dev(k_per_query, torch.int32, "k_per_query")
    npp = None if nprobe_per_query is None else _dev(nprobe_per_query, torch.int32, "nprobe_per_query")
    _check(lib().dade_search(ix.handle, qp, nq, k, nprobe, kp, npp, ctypes.byref(o),
                             _dev(out_ids, torch.int64, "out_ids"),
                             _dev(out_dist2, torch.float32, "out_dist2"), _stream(stream)))
    if record is not None:
        record.update(_record_dict(rec))
    return out_ids, out_dist2


def dade_search_noalloc(ix: Index, Q, k, nprobe, out_ids, out_dist2, k_per_query=None, nprobe_per_query=None,
                        delta_d=0, mode="dade", schedule="per_rank", rerank_delta=-1.0, stats=None, stream=None,
                        fill_min=32, growth=16, scan_blocks_per_cu=0, rerank_rule="all", record=None,
                        query_record=None):
    """dade_search without device allocation: the caller passes the output tensors ([nq, k] int64 and
    float32), the library works in its fixed per-device scratch.  Asynchronous."""
    import torch
    _search_args(ix, Q, k, out_ids, out_dist2, k_per_query, nprobe_per_query, stats, query_record)
    o = _search_opts(delta_d, mode, schedule, rerank_delta, fill_min, growth, False, scan_blocks_per_cu,
                     rerank_rule)
    o.stats = None if stats is None else _dev(stats, torch.int64, "stats").value
    o.query_record = None if query_record is None else _dev(query_record, torch.int32, "query_record").value
    rec = SearchRecord()
    if record is not None:
        o.record = ctypes.pointer(rec)
    kp = None if k_per_query is None else _dev(k_per_query, torch.int32, "k_per_query")
    npp = None if nprobe_per_query is None else _dev(nprobe_per_query, torch.int32, "nprobe_per_query")
    _check(lib().dade_search_noalloc(ix.handle, _dev(Q, torch.float32, "Q"), Q.shape[0], k, nprobe, kp, npp,
                                     ctypes.byref(o), _dev(out_ids, torch.int64, "out_ids"),
                                     _dev(out_dist2, torch.float32, "out_dist2"), _stream(stream)))
    if record is not None:
        record.update(_record_dict(rec))
    return out_ids, out_dist2


def _record_dict(rec):
    out = {name: getattr(rec, name) for name, _ in SearchRecord._fields_}
    out["mode"] = {v: k_ for k_, v in MODES.items()}[out["mode"]]
    out["schedule"] = {v: k_ for k_, v in SCHEDULES.items()}[out["schedule"]]
    out["rerank_rule"] = {v: k_ for k_, v in RERANK_RULES.items()}[out["rerank_rule"]]
    return out


def _search_opts(delta_d=0, mode="dade", schedule="per_rank", rerank_delta=-1.0, fill_min=32, growth=16,
                 use_graph=True, scan_blocks_per_cu=0, rerank_rule="all"):
    o = SearchOpts()
    o.delta_d, o.mode, o.schedule = delta_d, MODES[mode], SCHEDULES[schedule]
    o.rerank_delta = rerank_delta
    o.fill_min, o.growth = fill_min, growth
    o.use_graph, o.scan_blocks_per_cu = int(bool(use_graph)), scan_blocks_per_cu
    o.rerank_rule = RERANK_RULES[rerank_rule]
    return o


def dade_serve(ix: Index, arrival_s, req_queries, req_k, req_nprobe, Q, k_max, nprobe_max, budget_bytes=0,
               max_batch=0, max_inflight=0, stream=None, **search_kw):
    """Runs the serving loop over host request arrays and queries Q [sum(req_queries), dim] float32
    (a numpy array or a CPU torch tensor; pinned memory, e.g. ``torch.Tensor.pin_memory()``, is
    copied from directly); returns (ids [nq, k_max] int64, dist2 [nq, k_max] float32,
    latency_s [n_req], stats)."""
    if hasattr(Q, "is_pinned"):   # a CPU torch tensor: its memory as is
        if Q.is_cuda:
            raise TypeError("Q must be host memory")
        Q = Q.contiguous().numpy()
    arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
    nq = np.ascontiguousarray(req_queries, dtype=np.int32)
    ks = np.ascontiguousarray(req_k, dtype=np.int32)
    nps = np.ascontiguousarray(req_nprobe, dtype=np.int32)
    Qh = np.ascontiguousarray(Q, dtype=np.float32)
    n_req, total = len(arr), int(nq.sum()) if len(nq) else 0
    if not (len(nq) == len(ks) == len(nps) == n_req) or Qh.ndim != 2 or Qh.shape[0] != total:
        raise ValueError("request arrays must have one entry per request and Q one row per query")
    ids = np.empty((total, k_max), np.int64)
    d2 = np.empty((total, k_max), np.float32)
    lat = np.empty(n_req, np.float64)
    o = ServeOpts()
    o.budget_bytes, o.max_batch, o.max_inflight = budget_bytes, max_batch, max_inflight
    o.k_max, o.nprobe_max = k_max, nprobe_max
    o.search = _search_opts(**search_kw)
    st = ServeStats()
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    _check(lib().dade_serve(ix.handle, n_req, ptr(arr), ptr(nq), ptr(ks), ptr(nps), ptr(Qh), ctypes.byref(o),
                            ptr(ids), ptr(d2), ptr(lat), ctypes.byref(st), _stream(stream)))
    return ids, d2, lat, {name: getattr(st, name) for name, _ in ServeStats._fields_}


def dade_autotune(ix: Index, Q, k, nprobe, k_per_query=None, nprobe_per_query=None, min_agreement=0.0, reps=5,
                  stream=None, **search_kw):
    """Returns (chosen, table): `chosen` holds dade_search keyword arguments (delta_d, schedule,
    fill_min, growth, scan_blocks_per_cu) of the configuration picked; `table` one dict per
    configuration timed (its options, ms per search of Q and agreement with FULL_D)."""
    import torch
    o = _search_opts(**search_kw)
    kp = None if k_per_query is None else _dev(k_per_query, torch.int32, "k_per_query")
    npp = None if nprobe_per_query is None else _dev(nprobe_per_query, torch.int32, "nprobe_per_query")
    res = (TuneResult * TUNE_MAX)()
    n = ctypes.c_int32()
    _check(lib().dade_autotune(ix.handle, _dev(Q, torch.float32, "Q"), Q.shape[0], k, nprobe, kp, npp,
                               float(min_agreement), reps, ctypes.byref(o), res, ctypes.byref(n), _stream(stream)))
    names = {v: k_ for k_, v in SCHEDULES.items()}
    chosen = dict(delta_d=o.delta_d, schedule=names[o.schedule], fill_min=o.fill_min, growth=o.growth,
                  scan_blocks_per_cu=o.scan_blocks_per_cu)
    table = [dict(delta_d=r.delta_d, schedule=names[r.schedule], fill_min=r.fill_min, growth=r.growth,
                  scan_blocks_per_cu=r.scan_blocks_per_cu, ms=r.ms, agreement=r.agreement) for r in res[: n.value]]
    return chosen, table


def dade_graph_build(ix: Index, degree=16, reverse=8, nprobe=4, candidates=0, stream=None):
    _check(lib().dade_graph_build(ix.handle, degree, reverse, nprobe, candidates, _stream(stream)))


def dade_graph_search(ix: Index, Q, k, ef, n_entry=4, max_iters=0, delta_d=32, mode="dade", stats=None,
                      out_ids=None, out_dist2=None, stream=None):
    """Returns (ids [nq, k] int64, dist2 [nq, k] float32) device tensors (asynchronous)."""
    import torch
    nq = Q.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
    if out_dist2 is None:
        out_dist2 = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    o = _search_opts(delta_d=delta_d, mode=mode)
    o.stats = None if stats is None else _dev(stats, torch.int64, "stats").value
    _check(lib().dade_graph_search(ix.handle, _dev(Q, torch.float32, "Q"), nq, k, ef, n_entry, max_iters,
                                   ctypes.byref(o), _dev(out_ids, torch.int64, "out_ids"),
                                   _dev(out_dist2, torch.float32, "out_dist2"), _stream(stream)))
    return out_ids, out_dist2


def dade_graph_export(ix: Index):
    """(neighbors [n, width] int64 row ids, entries [nlist, 2] int64 row ids) on the host."""
    inf = dade_index_info(ix)
    deg = ctypes.c_int32()
    _check(lib().dade_graph_export(ix.handle, ctypes.byref(deg), None, None))
    nb = np.empty((inf["n"], deg.value), np.int64)
    en = np.empty((inf["nlist"], 2), np.int64)
    _check(lib().dade_graph_export(ix.handle, ctypes.byref(deg), ctypes.c_void_p(nb.ctypes.data),
                                   ctypes.c_void_p(en.ctypes.data)))
    return nb, en


def dade_check(ix: Index, stream=None):
    """Raises DadeError if a search on this index exceeded a list-scan capacity (synchronises)."""
    _check(lib().dade_check(ix.handle, _stream(stream)))


def dade_index_info(ix: Index):
    n, d, nl, st, state = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().dade_index_info(ix.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(nl),
                                 ctypes.byref(st), ctypes.byref(state)))
    return {"n": n.value, "dim": d.value, "nlist": nl.value, "store": st.value, "state": state.value}


def dade_export(ix: Index) -> dict:
    """Host copies (numpy) of the artifacts available in the index's state."""
    inf = dade_index_info(ix)
    n, dim, nl, state = inf["n"], inf["dim"], inf["nlist"], inf["state"]
    out = {"centroids": np.zeros((nl, dim)), "list_offsets": np.zeros(nl + 1, np.int64),
           "list_ids": np.zeros(n, np.int64)}
    if state >= STATE_ROTATED:
        out.update(W=np.zeros((dim, dim)), mu=np.zeros(dim), lam=np.zeros(dim))
    if state >= STATE_CALIBRATED:
        out["T"] = np.zeros(dim)
    a = Artifacts()
    ptr = lambda key: ctypes.c_void_p(out[key].ctypes.data) if key in out else None  # noqa: E731
    a.W, a.mu, a.lambda_, a.T = ptr("W"), ptr("mu"), ptr("lam"), ptr("T")
    a.centroids, a.list_offsets, a.list_ids = ptr("centroids"), ptr("list_offsets"), ptr("list_ids")
    _check(lib().dade_export(ix.handle, ctypes.byref(a)))
    out["delta"] = a.delta
    out.update(n=n, dim=dim, nlist=nl, state=state, store=inf["store"])
    return out


def dade_import(art: dict, X, store="f32", hbm_budget_bytes=0, stream=None) -> Index:
    """An index from host artifacts (keys: W, mu, lam, centroids, list_offsets, list_ids,
    optional T and delta) and the base vectors X (device)."""
    import torch
    keep = {k: np.ascontiguousarray(art[k], dtype=np.int64 if k.startswith("list") else np.float64)
            for k in ("W", "mu", "lam", "centroids", "list_offsets", "list_ids", "T") if art.get(k) is not None}
    a = Artifacts()
    a.n, a.dim, a.nlist = X.shape[0], X.shape[1], len(keep["list_offsets"]) - 1
    a.W, a.mu, a.lambda_ = (ctypes.c_void_p(keep[k].ctypes.data) for k in ("W", "mu", "lam"))
    a.T = ctypes.c_void_p(keep["T"].ctypes.data) if "T" in keep else None
    a.delta = float(art.get("delta", 0.0) or 0.0)
    a.centroids = ctypes.c_void_p(keep["centroids"].ctypes.data)
    a.list_offsets = ctypes.c_void_p(keep["list_offsets"].ctypes.data)
    a.list_ids = ctypes.c_void_p(keep["list_ids"].ctypes.data)
    o, _ = _build_opts(store, hbm_budget_bytes=hbm_budget_bytes)
    h = ctypes.c_void_p()
    _check(lib().dade_import(ctypes.byref(a), _dev(X, torch.float32, "X"), ctypes.byref(o), _stream(stream),
                             ctypes.byref(h)))
    return Index(h)


def dade_stage_times(ix: Index):
    t = Times()
    _check(lib().dade_stage_times(ix.handle, ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in Times._fields_}


def dade_destroy(ix: Index):
    ix.close()


def dade_last_error() -> str:
    return lib().dade_last_error().decode()
