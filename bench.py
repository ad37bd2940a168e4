"""Benchmark of the DADE-IVF search path on one MI355X.

Workload (default): 1M x 960 Gaussian mixture (2048 components, lam_i ~ i^-1.5), BF16 store
with FP32 rerank, 1000 queries, K = 10, nlist = 4096, Delta_d = 32.
A step is one dade_search of the whole query batch (query rotation, probe selection and the
list scan with top-K merge and rerank), inputs already resident in HBM.

The metric is QPS at recall@10 >= 0.95.  FDScanning (full-D exact DCOs) on the same index is
swept over nprobe; DADE over P_s (the significance level of the hypothesis test) and nprobe.
Each is timed at the fastest configuration reaching the target:
  * throughput: `--warmup` untimed searches, then `--steps` searches back to back between two
    device synchronisations (the list scan replays a captured HIP graph);
  * latency: `--steps` searches, each synchronised (p50 / p99);
  * kernel times: searches with HIP events around every kernel of the scan (launched without the
    graph), for the roofline of the DCO kernel.
Beside the metric (each leg can be skipped with its --no-* flag): the FP16 and FP32 stores on the
same lists, the data-oblivious transform, the linear scan, the serving loop under Poisson load
(p50 / p99 per request), an autotuner run, the graph search, and the CPU oracle baseline.
Other modes: --serving-only (a workload's request mix), --uneven-only (per-query K and nprobe in
one launch), --profile-only (timed steps only, for profilers).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPS at recall@10≥0.95, DADE vs full-D exact DCO, 1 GPU; p50/p99 latency"
PEAK_HBM_GBS = 8000.0
NPROBE_SWEEP = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256)
PS_SWEEP = (0.1, 0.05, 0.02, 0.01, 0.005, 0.002, 0.001, 0.0005)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ground_truth(torch, Xd, Qd, k, chunk=64):
    """Exact k nearest rows of every query (measurement only): FP64 squared distances on the GPU,
    ordered by (distance, id)."""
    X64 = Xd.double()
    xn = (X64 * X64).sum(1)
    out = []
    for s in range(0, Qd.shape[0], chunk):
        q = Qd[s:s + chunk].double()
        d2 = xn[None, :] - 2.0 * (q @ X64.T) + (q * q).sum(1, keepdim=True)
        d, i = torch.topk(d2, k + 8, dim=1, largest=False)
        d, i = d.cpu().numpy(), i.cpu().numpy()
        for r in range(len(d)):
            o = np.lexsort((i[r], d[r]))[:k]
            out.append(i[r][o])
    return np.stack(out).astype(np.int64)


def recall_at(ids, gt, k):
    hits = [len(set(ids[i, :k].tolist()) & set(gt[i, :k].tolist())) for i in range(len(gt))]
    return float(np.mean(hits)) / k


def scan_source_sha(src=None):
    """Hash of the DCO kernel's sources with comments and blank lines left out (a comment edit
    does not invalidate the counters)."""
    h = hashlib.sha256()
    for f in ("scan.hip", "kernels.h", "common.h"):
        text = src[f] if src else open(os.path.join(ROOT, "paper_2411_17229_amd", "csrc", f)).read()
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_from_profile(workload, store, nprobe, p_s):
    """HBM bytes per DCO-kernel launch from the committed rocprofv3 counter summary, if it was taken
    on the current scan source at the same operating point and round schedule; else None."""
    path = os.path.join(ROOT, "profiles", "scan_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    e = rec.get(f"{workload}/{store}/nprobe{nprobe}/p_s{p_s}/{SCHEDULE['schedule']}/fill{SCHEDULE['fill_min']}"
                f"/growth{SCHEDULE['growth']}")
    if not e or e.get("scan_sha") != scan_source_sha():
        return None
    return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


SCHEDULE = dict(schedule="whole", fill_min=32, growth=0)   # round schedule of the timed runs: the fill round, then the rest


def throughput(dade, torch, ix, Qd, k, nprobe, steps, warmup, **kw):
    """`warmup` untimed searches, then exactly `steps` searches back to back, bracketed by
    device synchronisation; returns ms per step."""
    for _ in range(warmup):
        dade.dade_search(ix, Qd, k, nprobe, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dade.dade_search(ix, Qd, k, nprobe, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def latencies(dade, torch, ix, Qd, k, nprobe, steps, **kw):
    """Wall time of each search from enqueue to completion (one batch at a time)."""
    walls = []
    for _ in range(steps):
        t0 = time.perf_counter()
        dade.dade_search(ix, Qd, k, nprobe, **kw)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    return np.array(walls)


def kernel_times(dade, torch, ix, Qd, k, nprobe, steps, **kw):
    """Per-stage and per-kernel times (HIP events on the kernels' stream), averaged over steps."""
    acc = {}
    for _ in range(steps):
        dade.dade_search(ix, Qd, k, nprobe, record_times=True, **kw)
        for key, v in dade.dade_stage_times(ix).items():
            acc[key] = acc.get(key, 0.0) + v
    return {key: v / steps for key, v in acc.items()}


def _oracle_index(art, X, store):
    """The oracle's view of the library's index (its lists, W, mu, lambda, T and delta, exported):
    stored rows rotated on demand from X (and rounded as the store rounds them), exact rows for
    the low-precision rerank."""
    from oracle import estimator, ivf, lowp
    lam, T = art["lam"], art["T"]
    eps = np.sqrt(np.maximum(T * estimator.scale(lam), 0.0)) - 1.0
    rnd = None if store == "f32" else (lambda y: lowp.store(y, store))
    Y = ivf.LazyRotated(X, art["mu"], art["W"], rnd)
    Ye = ivf.LazyRotated(X, art["mu"], art["W"]) if rnd is not None else None
    return ivf.Index(art["mu"], art["W"], lam, eps, art["centroids"], art["list_offsets"], art["list_ids"], Y,
                     Y_exact=Ye, delta=art["delta"], T=T)


CPU_ART_KEYS = ("W", "mu", "lam", "T", "centroids", "list_offsets", "list_ids")


def cpu_baseline(w, X, Q, art, store, nprobe, p_s, rerank, gt, seconds=20.0):
    """The FP64 oracle timed on the host on a bounded sample of the workload itself: the library's
    index (exported lists, transform, thresholds and rerank margin; rows rotated on demand), the
    timed runs' schedule, nprobe, P_s and rerank rule, queries in order until ~`seconds`; the rate is
    extrapolated from that query subsample.  One thread (BLAS limited to one), the same in exact
    mode (FDScanning) for half the time, and every usable core in a child process.  Beside it, not
    timed: the round schedule against the paper's sequential one (heap updated after every DCO) on
    a query sample, recall@K against FP64 brute force and dimensions read."""
    from threadpoolctl import threadpool_limits

    from oracle import ivf
    oi = _oracle_index(art, X, store)
    kw = dict(SCHEDULE, rerank=rerank)

    def timed(mode, budget):
        with threadpool_limits(limits=1):
            done, t0 = 0, time.perf_counter()
            while done < len(Q) and time.perf_counter() - t0 < budget:
                ivf.search(oi, Q[done:done + 1], w.k, nprobe, w.delta_d, mode=mode, **kw)
                done += 1
            return done, time.perf_counter() - t0

    done, el = timed("dade", seconds)
    out = {"value": done / el, "unit": "queries/s", "cores": 1, "kind": "oracle",
           "sample": f"the first {done} of the workload's {len(Q)} queries (rate extrapolated) on the library's "
                     f"{w.n} x {w.dim} index (exported lists, W, T and delta; {store} rows rotated on demand "
                     f"from X), DADE, {SCHEDULE['schedule']} rounds, P_s {p_s}, nprobe {nprobe}, K {w.k}, "
                     f"rerank rule {rerank}; one thread (BLAS limited to one)"}
    done_f, el_f = timed("full_d", seconds / 2)
    out["full_d"] = {"value": done_f / el_f, "unit": "queries/s", "cores": 1, "kind": "oracle",
                     "sample": f"the first {done_f} queries, FULL_D mode (FDScanning), same index, nprobe and K; "
                               f"one thread"}
    # the same search on every usable core: a child process (this one holds the GPU) regenerates
    # the workload, loads the exported artifacts and forks one single-threaded worker per core
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "index.npz")
        np.savez(path, **{k_: art[k_] for k_ in CPU_ART_KEYS}, delta=np.array(art["delta"]))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-pool", path, "--workload", w.name,
                            "--store", store, "--nprobe", str(nprobe), "--p-s", str(p_s), "--rerank", rerank,
                            "--schedule", SCHEDULE["schedule"],
                            "--cpu-seconds", str(seconds)], capture_output=True, text=True, timeout=900)
    if r.returncode == 0 and r.stdout.strip():
        out["all_cores"] = json.loads(r.stdout.strip().splitlines()[-1])
    else:
        out["all_cores"] = {"error": (r.stderr or "")[-300:]}
    out["schedule_gap"] = schedule_gap(oi, w, Q, gt, nprobe, rerank)
    return out


def schedule_gap(oi, w, Q, gt, nprobe, rerank, n_sample=20):
    """The round schedule's snapshots against the paper's sequential heap (one candidate per round)
    in the oracle: recall@K and the fraction of dimensions read on the first queries."""
    from oracle import ivf
    out = {"queries": n_sample, "nprobe": nprobe}
    for name, kw in (("rounds", dict(SCHEDULE)), ("sequential", dict(schedule="sequential"))):
        t0 = time.perf_counter()
        ids, _, logs = ivf.search(oi, Q[:n_sample], w.k, nprobe, w.delta_d, log=True, rerank=rerank, **kw)
        out[name] = {"recall@%d" % w.k: round(recall_at(ids, gt[:n_sample], w.k), 4),
                     "dims_frac": round(float(logs["dims"].sum()) / float(logs["dcos"].sum() * w.dim), 5),
                     "oracle_s": round(time.perf_counter() - t0, 1)}
    log(f"[bench] schedule gap: {out}")
    return out


def oracle_pool(path, w, store, nprobe, p_s, rerank, seconds):
    """Child of cpu_baseline (no GPU here): the workload regenerated, the oracle's view of the exported
    index, then one single-threaded worker per usable core (at most 16) searching every P-th query
    for ~`seconds`."""
    import multiprocessing as mp

    from paper_2411_17229_amd import workloads
    d = np.load(path)
    art = {k_: d[k_] for k_ in CPU_ART_KEYS}
    art["delta"] = float(d["delta"])
    X, Q = workloads.make(w)
    global _POOL_INDEX
    _POOL_INDEX = (_oracle_index(art, X, store), Q, w, nprobe, rerank, seconds)
    cores = min(16, len(os.sched_getaffinity(0)))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        counts = pool.map(_pool_worker, [(i, cores) for i in range(cores)])
    el = time.perf_counter() - t0
    return {"value": sum(counts) / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{sum(counts)} queries over {cores} single-threaded worker processes, same index and "
                      f"settings as the one-thread run (rate extrapolated); wall time includes the pool's start"}


def _pool_worker(arg):
    from threadpoolctl import threadpool_limits

    from oracle import ivf
    i, cores = arg
    oi, Q, w, nprobe, rerank, seconds = _POOL_INDEX
    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        for qi in range(i, len(Q), cores):
            if time.perf_counter() - t0 >= seconds:
                break
            ivf.search(oi, Q[qi:qi + 1], w.k, nprobe, w.delta_d, rerank=rerank, **SCHEDULE)
            done += 1
    return done


ABL_PS = (0.3, 0.2, 0.1, 0.05, 0.02, 0.01, 0.005)   # P_s of the data-oblivious comparison


def oblivious_ablation(dade, torch, ix, Xd, Qd, w, gt, store, pairs, nprobe, steps):
    """The data-aware transform against a seeded data-oblivious one (the random orthogonal
    projection of Figure 1): the same lists, store, schedule and calibration pairs; recall@10,
    fraction of dimensions read and QPS over P_s, and the variance each captures in its first d
    dimensions.  Leaves ix calibrated at the last P_s."""
    from paper_2411_17229_amd import workloads
    nq = Qd.shape[0]
    art = dade.dade_export(ix)
    W_r = workloads.oblivious_rotation(w.dim, w.seed)
    # variance along each random axis, from the data-aware eigendecomposition (reported only;
    # the test uses the calibrated T_d)
    lam_r = ((art["W"].T @ W_r) ** 2 * art["lam"][:, None]).sum(0)
    keep = {k: v for k, v in art.items() if k not in ("T", "delta", "W", "lam")}
    rop = dade.dade_import({**keep, "W": W_r, "lam": lam_r}, Xd, store=store)
    out = {"transform": "seeded Haar rotation", "nprobe": nprobe, "delta_d": w.delta_d,
           "variance_frac": {}, "by_p_s": {}}
    for name, lam in (("data_aware", art["lam"]), ("oblivious", lam_r)):
        c = np.cumsum(lam) / lam.sum()
        out["variance_frac"][name] = {str(dd): round(float(c[dd - 1]), 4) for dd in (32, 64, 128, 256, w.dim // 2)}
    for ps in ABL_PS:
        row = {}
        for name, index in (("data_aware", ix), ("oblivious", rop)):
            dade.dade_calibrate(index, ps, pairs=pairs)
            stats = torch.zeros((nq, 4), dtype=torch.int64, device=Qd.device)
            ids, _ = dade.dade_search(index, Qd, w.k, nprobe, stats=stats, delta_d=w.delta_d, **SCHEDULE)
            torch.cuda.synchronize()
            dade.dade_check(index)
            st = stats.cpu().numpy().sum(0)
            ms = throughput(dade, torch, index, Qd, w.k, nprobe, steps, 2, delta_d=w.delta_d, **SCHEDULE)
            row[name] = {"recall@10": round(recall_at(ids.cpu().numpy(), gt, w.k), 4),
                         "dims_frac": round(float(st[1]) / max(1, st[0] * w.dim), 4),
                         "qps": round(nq / (ms / 1e3), 1)}
        out["by_p_s"][str(ps)] = row
        log(f"[bench] ablation P_s {ps}: {row}")
    rop.close()
    return out


LIN_DD = (1, 2, 4, 8, 16, 32, 64)   # Delta_d of the linear-scan study
LIN_SCHEDULE = dict(schedule="doubling", fill_min=32, growth=16)   # growth-capped rounds tighten r inside the one list
# the uneven batch's P_s sweep and FDScanning runs (nprobe up to 128): the doubling schedule, as
# in every run of this study that completed
UNEVEN_SCHEDULE = dict(schedule="doubling", fill_min=32, growth=0)


def linear_scan(dade, torch, w, store, p_s, steps, n=100_000, nq=200):
    """Linear-scan feasibility (one list holds every row, so every query scans all n rows): DADE
    at each Delta_d against FDScanning on the same index; recall@10, fraction of dimensions read
    and QPS.  Rows and queries come from the workload's generator (its first n rows)."""
    from paper_2411_17229_amd import workloads
    X, Q = workloads.make(w, n=n, n_queries=nq)
    Xd, Qd = torch.from_numpy(X).to("cuda:0"), torch.from_numpy(Q).to("cuda:0")
    ix = dade.dade_build_index(Xd, 1, store=store, init_rows=np.zeros(1, np.int64))
    dade.dade_rotate(ix)
    dade.dade_calibrate(ix, p_s, pairs=workloads.calibration_pairs(n, 100_000, w.seed))
    gt = ground_truth(torch, Xd, Qd, w.k)
    out = {"n": n, "dim": w.dim, "queries_per_step": nq, "store": store, "p_s": p_s, "nlist": 1,
           "schedule": LIN_SCHEDULE, "by_delta_d": {}}
    for mode, dds in (("full_d", (w.delta_d,)), ("dade", LIN_DD)):
        for dd in dds:
            stats = torch.zeros((nq, 4), dtype=torch.int64, device=Qd.device)
            ids, _ = dade.dade_search(ix, Qd, w.k, 1, stats=stats, delta_d=dd, mode=mode, **LIN_SCHEDULE)
            torch.cuda.synchronize()
            dade.dade_check(ix)
            st = stats.cpu().numpy().sum(0)
            ms = throughput(dade, torch, ix, Qd, w.k, 1, steps, 1, delta_d=dd, mode=mode, **LIN_SCHEDULE)
            row = {"recall@10": round(recall_at(ids.cpu().numpy(), gt, w.k), 4),
                   "dims_frac": round(float(st[1]) / max(1, st[0] * w.dim), 4), "qps": round(nq / (ms / 1e3), 1)}
            if mode == "full_d":
                out["full_d"] = row
            else:
                out["by_delta_d"][str(dd)] = row
            log(f"[bench] linear scan {mode} delta_d {dd}: {row}")
    ix.close()
    return out


SERVE_RATES = (0.25, 0.5, 0.75, 0.9, 1.0, 1.1)


def serving_sweep(dade, ix, Q, gt, k, ks, nprobes, n_req=2000, budget=512 << 20, max_batch=2048, seed=0, **kw):
    """The serving loop (dade_serve): its saturated throughput (every request arriving at once),
    then Poisson arrivals at fractions of it: per offered rate, achieved QPS, p50/p99 request latency (arrival to results on
    the host) and recall@k of the served rows.  Requests hold 1..256 queries (log-uniform) with
    K and nprobe drawn from `ks` x `nprobes`; their queries cycle through Q and are handed over in
    pinned host memory (a serving front end's receive buffers), which the loop copies from."""
    import torch

    from paper_2411_17229_amd import workloads
    _, sizes, rk, rn = workloads.requests(n_req, 1.0, ks=ks, nprobes=nprobes, seed=seed)
    sizes = sizes.astype(np.int32)
    total = int(sizes.sum())
    rows = np.arange(total) % len(Q)
    Qs = torch.from_numpy(Q[rows]).pin_memory()
    k_max, np_max = int(max(ks)), int(max(nprobes))
    # warm-up (allocations, code objects); then the saturated throughput: every request arrives
    # at once; then one run per offered rate (sizes, K and nprobe do not depend on the rate: the
    # gaps are drawn first and scaled by it)
    dade.dade_serve(ix, np.zeros(8), sizes[:8], rk[:8], rn[:8], Q[rows[: int(sizes[:8].sum())]], k_max, np_max,
                    budget_bytes=budget, max_batch=max_batch, **kw)
    bursts = [dade.dade_serve(ix, np.zeros(n_req), sizes, rk, rn, Qs, k_max, np_max, budget_bytes=budget,
                              max_batch=max_batch, **kw)[3] for _ in range(2)]   # the first pays one-time costs
    st = min(bursts, key=lambda b: b["wall_s"])
    sat_qps = st["served_queries"] / st["wall_s"]
    burst = {"qps": round(sat_qps, 1), "wall_ms": round(st["wall_s"] * 1e3, 3), "launches": st["launches"],
             "mean_queries_per_launch": round(st["served_queries"] / max(1, st["launches"]), 1)}
    log(f"[bench] serving burst: {sat_qps:.0f} QPS over {st['launches']} launches")
    out = []
    for f in SERVE_RATES:
        rate_rps = f * sat_qps / sizes.mean()
        arr = workloads.requests(n_req, rate_rps, ks=ks, nprobes=nprobes, seed=seed)[0]
        ids, _, lat, st = dade.dade_serve(ix, arr, sizes, rk, rn, Qs, k_max, np_max, budget_bytes=budget,
                                          max_batch=max_batch, **kw)
        served = lat >= 0
        rec = recall_at(ids[:, :k], gt[rows], k)
        out.append({"offered_fraction": f, "offered_qps": round(f * sat_qps, 1),
                    "achieved_qps": round(st["served_queries"] / st["wall_s"], 1),
                    "p50_ms": round(float(np.percentile(lat[served], 50)) * 1e3, 4),
                    "p99_ms": round(float(np.percentile(lat[served], 99)) * 1e3, 4),
                    "mean_queries_per_launch": round(st["served_queries"] / max(1, st["launches"]), 1),
                    "waited_requests": st["waited_requests"], "rejected_requests": st["rejected_requests"],
                    "host_ms": {"stage": round(st["stage_s"] * 1e3, 3), "launch": round(st["launch_s"] * 1e3, 3),
                                "retire": round(st["retire_s"] * 1e3, 3)},
                    "recall@%d" % k: round(rec, 4)})
        log(f"[bench] serving at {f:.2f} x {sat_qps:.0f} QPS: {out[-1]['achieved_qps']:.0f} QPS, "
            f"p50 {out[-1]['p50_ms']:.3f} ms, p99 {out[-1]['p99_ms']:.3f} ms, "
            f"{out[-1]['mean_queries_per_launch']} queries/launch, recall {rec:.4f}")
    return {"requests_per_rate": n_req, "queries_per_rate": total, "mean_request_queries": round(float(sizes.mean()), 2),
            "k": list(map(int, ks)), "nprobe": list(map(int, nprobes)), "ring_slots": st["ring_slots"],
            "workspace_bytes": st["workspace_bytes"], "budget_bytes": budget, "max_batch": max_batch,
            "pinned_queries": True, "saturated": burst, "rates": out}


GRAPH_EF = (16, 32, 64)
GRAPH_ENTRY = (2, 4, 16)


GRAPH_BUILDS = {   # name -> (out-degree, back links, candidates (0: the plain kNN graph), build nprobe (None: all lists))
    "knn": (16, 8, 0, 4),
    "hnsw_select": (16, 16, 64, None),
}


def graph_study(dade, torch, target, steps, sample=None):
    """The graph setting (a one-layer graph, DADE DCOs in a beam search), on rows of at most
    20,000 (the graph build's limit): the 20k x 128 workload, or with `sample` = (workload, X, Q,
    P_s) the first 20,000 rows of that workload (iid draws of its mixture) with nlist scaled to
    keep its list size.  Two builds (GRAPH_BUILDS): the plain kNN graph from an FDScanning search
    over 4 lists, and HNSW's neighbour selection over each row's 64 nearest from a search over all
    lists (the exact nearest rows).  Per build its time, then per (entry lists, ef) the recall@k,
    QPS and dimensions read of DADE and FDScanning; the headline pair is each mode's fastest
    setting, over both builds, reaching `target`.  A search runs at most 2 ef expansions, fewer
    where the visited table's bound (2 n_entry + expansions x row width <= 4096) asks for it."""
    import dataclasses as dc

    from paper_2411_17229_amd import workloads
    if sample is None:
        w = workloads.WORKLOADS["small-20k-d128"]
        X, Q = workloads.make(w, n_queries=1000)
        p_s = w.alpha
    else:
        w0, X0, Q, p_s = sample
        n = 20_000
        X = np.ascontiguousarray(X0[:n])
        w = dc.replace(w0, name=f"{w0.name}-first{n}", n=n, nlist=max(1, round(w0.nlist * n / w0.n)))
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    store = w.store
    ix = dade.dade_build_index(Xd, w.nlist, store=store, init_rows=workloads.kmeans_init_rows(w.n, w.nlist, w.seed))
    dade.dade_rotate(ix)
    dade.dade_calibrate(ix, p_s, pairs=workloads.calibration_pairs(w.n, 100_000, w.seed))
    gt = ground_truth(torch, Xd, Qd, w.k)
    nq = Qd.shape[0]
    s_bytes = 2 if store in ("bf16", "f16") else 4
    out = {"workload": w.name, "n": w.n, "dim": w.dim, "nlist": w.nlist, "queries": len(Q), "p_s": p_s, "store": store,
           "builds": {}}
    best = {}
    for name, (degree, reverse, candidates, nprobe_build) in GRAPH_BUILDS.items():
        nprobe_build = nprobe_build or w.nlist
        t0 = time.perf_counter()
        dade.dade_graph_build(ix, degree=degree, reverse=reverse, nprobe=nprobe_build, candidates=candidates)
        build_s = time.perf_counter() - t0
        bo = {"degree": degree, "reverse": reverse, "candidates": candidates, "nprobe_build": nprobe_build,
              "build_s": round(build_s, 2), "sweep": {}}
        log(f"[bench] graph {name}: degree {degree} (candidates {candidates}) + {reverse} back links, build nprobe "
            f"{nprobe_build}, built in {build_s:.1f}s")
        for mode in ("dade", "full_d"):
            rows = {}
            for n_entry, ef in [(e, f) for e in GRAPH_ENTRY for f in GRAPH_EF]:
                iters = min(2 * ef, (4096 - 2 * n_entry) // (degree + reverse))
                kw = dict(n_entry=n_entry, delta_d=w.delta_d, mode=mode, max_iters=iters)
                stats = torch.zeros((nq, 4), dtype=torch.int64, device=Qd.device)
                ids, _ = dade.dade_graph_search(ix, Qd, w.k, ef, stats=stats, **kw)
                torch.cuda.synchronize()
                st = stats.cpu().numpy().sum(0)
                rec = recall_at(ids.cpu().numpy(), gt, w.k)
                for _ in range(2):
                    dade.dade_graph_search(ix, Qd, w.k, ef, **kw)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                e0.record()
                for _ in range(steps):
                    dade.dade_graph_search(ix, Qd, w.k, ef, **kw)
                e1.record()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / steps
                r_ = {"recall@10": round(rec, 4), "qps": round(nq / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                      "event_ms": round(e0.elapsed_time(e1) / steps, 4),
                      "dcos_per_query": round(float(st[0]) / nq, 1),
                      "dims_frac": round(float(st[1]) / max(1, st[0] * w.dim), 4),
                      "steps_per_query": round(float(st[2]) / nq, 1), "max_iters": iters,
                      "alg_GBps": round(s_bytes * float(st[1]) / (ms * 1e-3) / 1e9, 1)}
                rows[(n_entry, ef)] = r_
                log(f"[bench] graph {name} {mode} entry {n_entry} ef {ef}: recall {rec:.4f} {r_['qps']:.0f} QPS "
                    f"dims {r_['dims_frac']:.4f} dcos/q {r_['dcos_per_query']}")
                cur = best.get(mode)
                key = (rec >= target, r_["qps"] if rec >= target else rec)
                if cur is None or key > cur[0]:
                    best[mode] = (key, dict(build=name, n_entry=n_entry, ef=ef, **r_))
            bo["sweep"][mode] = {f"entry{k_[0]}_ef{k_[1]}": v for k_, v in rows.items()}
        out["builds"][name] = bo
    for mode in ("dade", "full_d"):
        out[mode] = best[mode][1]
    out["speedup_vs_full_d"] = round(out["dade"]["qps"] / out["full_d"]["qps"], 3)
    ix.close()
    return out


def uneven_study(dade, torch, ix, Xd, Qd, w, store, target, steps, warmup):
    """One launch of the uneven batch (per-query K and nprobe drawn as the workload states): P_s is
    the largest of the sweep whose mean recall@K reaches `target`; Delta_d and the round and launch
    shapes come from the autotuner (first 512 queries, agreement bound `target`); then DADE and
    FDScanning are timed on the whole batch, with recall@K per K."""
    from paper_2411_17229_amd import workloads
    nq = Qd.shape[0]
    K, npb = workloads.uneven_batch(nq, 8, 128, (1, 10, 50, 100), seed=w.seed)
    kp, npp = torch.from_numpy(K).to(Qd.device), torch.from_numpy(npb).to(Qd.device)
    kmax, npmax = int(K.max()), int(npb.max())
    gt = ground_truth(torch, Xd, Qd, kmax)
    pairs = workloads.calibration_pairs(w.n, 100_000, w.seed)

    def recall(ids):
        r = np.array([len(set(ids[i, :K[i]].tolist()) & set(gt[i, :K[i]].tolist())) / K[i] for i in range(nq)])
        return float(r.mean()), {str(k_): round(float(r[K == k_].mean()), 4) for k_ in sorted(set(K.tolist()))}

    base = dict(delta_d=w.delta_d, **UNEVEN_SCHEDULE)
    by_ps = {}
    chosen_ps = PS_SWEEP[-1]
    for ps in PS_SWEEP:
        dade.dade_calibrate(ix, ps, pairs=pairs)
        ids, _ = dade.dade_search(ix, Qd, kmax, npmax, k_per_query=kp, nprobe_per_query=npp, **base)
        by_ps[str(ps)] = round(recall(ids.cpu().numpy())[0], 4)
        log(f"[bench] uneven: P_s {ps} recall {by_ps[str(ps)]}")
        if by_ps[str(ps)] >= target:
            chosen_ps = ps
            break
    dade.dade_calibrate(ix, chosen_ps, pairs=pairs)
    tuned, table = dade.dade_autotune(ix, Qd[:512].contiguous(), kmax, npmax, k_per_query=kp[:512].contiguous(),
                                      nprobe_per_query=npp[:512].contiguous(), min_agreement=target, reps=3)
    log(f"[bench] uneven: autotuned {tuned}")
    out = {"workload": w.name, "n": w.n, "dim": w.dim, "nlist": w.nlist, "store": store, "queries": nq,
           "k_mix": {str(k_): int((K == k_).sum()) for k_ in sorted(set(K.tolist()))},
           "nprobe_mean": round(float(npb.mean()), 1), "p_s": chosen_ps, "recall_by_p_s": by_ps, "autotuned": tuned}
    for mode, kw in (("dade", dict(tuned)), ("full_d", dict(base, mode="full_d"))):
        ms = throughput(dade, torch, ix, Qd, kmax, npmax, steps, warmup, k_per_query=kp, nprobe_per_query=npp, **kw)
        record = {}
        ids, _ = dade.dade_search(ix, Qd, kmax, npmax, k_per_query=kp, nprobe_per_query=npp, record=record, **kw)
        rec, per_k = recall(ids.cpu().numpy())
        out[mode] = {"qps": round(nq / (ms / 1e3), 1), "ms_per_step": round(ms, 4), "recall": round(rec, 4),
                     "recall_by_k": per_k, "search_record": record}
        log(f"[bench] uneven {mode}: {out[mode]['qps']:.0f} QPS ({ms:.3f} ms per batch), recall {rec:.4f} {per_k}")
    out["speedup_vs_full_d"] = round(out["dade"]["qps"] / out["full_d"]["qps"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="highd-1m-d960")
    ap.add_argument("--store", default=None)
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--k", type=int, default=None, help="K of every query (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the data-aware vs data-oblivious transform comparison")
    ap.add_argument("--no-linear", action="store_true", help="skip the linear-scan (one list) study")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop sweep")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner run")
    ap.add_argument("--no-graph-study", action="store_true", help="skip the graph-search study")
    ap.add_argument("--uneven-only", action="store_true",
                    help="build, then only measure the workload's uneven batch (per-query K in {1, 10, 50, 100}, "
                         "nprobe in 8..128): DADE with autotuned options against FDScanning")
    ap.add_argument("--serving-only", action="store_true",
                    help="build, then only run the serving-loop sweep with the workload's request mix "
                         "(K in {10, 100}, nprobe in {32, 96}) at --p-s")
    ap.add_argument("--serve-budget-mib", type=int, default=None,
                    help="device budget of the serving loop (default 512 MiB; 4 GiB with --serving-only)")
    ap.add_argument("--profile-only", action="store_true",
                    help="build, then only run timed DADE steps at --nprobe / --p-s (for profilers)")
    ap.add_argument("--nprobe", type=int, default=None)
    ap.add_argument("--p-s", type=float, default=None)
    ap.add_argument("--mode", default="dade")
    ap.add_argument("--schedule", default=SCHEDULE["schedule"], choices=("per_rank", "doubling", "whole"),
                    help="round schedule of the timed runs (fill 32, no growth cap)")
    ap.add_argument("--rerank", default="lazy", choices=("all", "lazy"),
                    help="low-precision rerank rule of the timed runs: every survivor that passes the gate, or "
                         "the lazy rule (the default; the other rule is timed beside it)")
    ap.add_argument("--no-graph", action="store_true",
                    help="with --profile-only: launch the scan kernels one by one (counter collection "
                         "does not see kernels replayed from a graph)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    ap.add_argument("--oracle-pool", default=None, help=argparse.SUPPRESS)   # child of the CPU baseline
    args = ap.parse_args()
    SCHEDULE["schedule"] = args.schedule
    if args.oracle_pool:
        from paper_2411_17229_amd import workloads
        print(json.dumps(oracle_pool(args.oracle_pool, workloads.WORKLOADS[args.workload], args.store, args.nprobe,
                                     args.p_s, args.rerank, args.cpu_seconds)), flush=True)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 5 copies of {src.numel() * 4} bytes")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_17229_amd import dade, workloads
    w = workloads.WORKLOADS[args.workload]
    if args.k:
        w = dataclasses.replace(w, k=args.k)
    store = args.store or w.store
    t0 = time.perf_counter()
    X, Q = workloads.make(w)
    log(f"[bench] data {X.shape} + {Q.shape} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    Xd, Qd = torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev)
    t0 = time.perf_counter()
    ix = dade.dade_build_index(Xd, w.nlist, store=store, init_rows=workloads.kmeans_init_rows(w.n, w.nlist, w.seed))
    t_build = time.perf_counter() - t0
    dade.dade_rotate(ix)
    t_rot = time.perf_counter() - t0 - t_build
    dade.dade_calibrate(ix, args.p_s or w.alpha, pairs=workloads.calibration_pairs(w.n, 100_000, w.seed))
    t_cal = time.perf_counter() - t0 - t_build - t_rot
    log(f"[bench] index: k-means {t_build:.1f}s, transform {t_rot:.1f}s, calibrate {t_cal:.1f}s")
    nq = Qd.shape[0]

    if args.profile_only:
        npb = args.nprobe or w.nprobe
        kw = dict(delta_d=w.delta_d, mode=args.mode, use_graph=not args.no_graph, rerank_rule=args.rerank, **SCHEDULE)
        ms = throughput(dade, torch, ix, Qd, w.k, npb, args.steps, args.warmup, **kw)
        log(f"[bench] profile run ({args.mode}, nprobe {npb}, P_s {args.p_s or w.alpha}): {ms:.3f} ms/step")
        return

    t0 = time.perf_counter()
    gt = ground_truth(torch, Xd, Qd, w.k)
    log(f"[bench] FP64 ground truth in {time.perf_counter() - t0:.1f}s")

    if args.uneven_only:
        print(json.dumps(uneven_study(dade, torch, ix, Xd, Qd, w, store, args.target, args.steps, args.warmup)),
              flush=True)
        return

    if args.serving_only:
        # P_s: the largest of the sweep whose recall@10 at the mix's smaller nprobe reaches the target
        # (unless --p-s fixes it)
        pairs = workloads.calibration_pairs(w.n, 100_000, w.seed)
        chosen_ps, rec_by_ps = args.p_s, {}
        for ps in ([args.p_s] if args.p_s else PS_SWEEP):
            dade.dade_calibrate(ix, ps, pairs=pairs)
            ids, _ = dade.dade_search(ix, Qd, w.k, 32, delta_d=w.delta_d, **SCHEDULE)
            rec_by_ps[str(ps)] = round(recall_at(ids.cpu().numpy(), gt, w.k), 4)
            log(f"[bench] serving workload: P_s {ps} recall@10 at nprobe 32: {rec_by_ps[str(ps)]}")
            chosen_ps = ps
            if rec_by_ps[str(ps)] >= args.target:
                break
        mib = args.serve_budget_mib or 4096
        sv = serving_sweep(dade, ix, Q, gt, w.k, (10, 100), (32, 96), budget=mib << 20, seed=w.seed,
                           delta_d=w.delta_d, **SCHEDULE)
        print(json.dumps({"workload": w.name, "n": w.n, "dim": w.dim, "nlist": w.nlist, "store": store,
                          "p_s": chosen_ps, "recall@10_nprobe32_by_p_s": rec_by_ps, "delta_d": w.delta_d,
                          "schedule": SCHEDULE, "serving": sv}), flush=True)
        return

    pairs = workloads.calibration_pairs(w.n, 100_000, w.seed)
    RR = dict(rerank_rule=args.rerank)

    def first_reaching(mode, kw):
        """(nprobe, recall, curve): smallest swept nprobe with recall >= target (else best)."""
        curve = {}
        for npb in NPROBE_SWEEP:
            if npb > w.nlist:
                break
            ids, _ = dade.dade_search(ix, Qd, w.k, npb, delta_d=w.delta_d, mode=mode, **kw, **RR)
            torch.cuda.synchronize()
            curve[npb] = recall_at(ids.cpu().numpy(), gt, w.k)
            if curve[npb] >= args.target:
                return npb, curve[npb], curve
            if len(curve) >= 3 and curve[npb] <= list(curve.values())[-3] + 1e-4:
                break   # recall has stopped growing with nprobe
        best = max(curve, key=lambda p: curve[p])
        return best, curve[best], curve

    # operating points (untimed sweeps), each method at its own fastest configuration reaching the
    # target: full-D at its smallest such nprobe (its work grows with nprobe); DADE over (P_s, the
    # smallest nprobe reaching the target at that P_s), the fastest of those timed
    sweep = {"full_d": {}, "dade": {}}
    chosen = {}
    npb, r, sweep["full_d"] = first_reaching("full_d", SCHEDULE)
    chosen["full_d"] = (None, npb, r)
    log(f"[bench] full_d: nprobe {npb} recall {r:.4f}")
    cands = []
    for ps in PS_SWEEP:
        dade.dade_calibrate(ix, ps, pairs=pairs)
        npb, r, curve = first_reaching("dade", SCHEDULE)
        sweep["dade"][str(ps)] = curve
        log(f"[bench] dade P_s {ps}: nprobe {npb} recall {r:.4f}")
        if r >= args.target:
            ms = throughput(dade, torch, ix, Qd, w.k, npb, 5, 2, delta_d=w.delta_d, **SCHEDULE, **RR)
            cands.append((ms, ps, npb, r))
    if cands:
        _, ps, npb, r = min(cands)
    else:
        ps = PS_SWEEP[-1]
        npb = max(sweep["dade"][str(ps)], key=lambda p: sweep["dade"][str(ps)][p])
        r = sweep["dade"][str(ps)][npb]
    chosen["dade"] = (ps, npb, r)
    dade.dade_calibrate(ix, ps, pairs=pairs)
    s_bytes = 2 if store in ("bf16", "f16") else 4
    res = {}
    for mode in ("dade", "full_d"):
        ps_m, npb, r_m = chosen[mode]
        kw = dict(delta_d=w.delta_d, mode=mode, **SCHEDULE, **RR)
        stats = torch.zeros((nq, 4), dtype=torch.int64, device=dev)
        rec = {}
        ids, d2 = dade.dade_search(ix, Qd, w.k, npb, stats=stats, record=rec, **kw)
        torch.cuda.synchronize()
        dade.dade_check(ix)
        st = stats.cpu().numpy().sum(0)
        ms = throughput(dade, torch, ix, Qd, w.k, npb, args.steps, args.warmup, **kw)
        walls = latencies(dade, torch, ix, Qd, w.k, npb, args.steps, **kw)
        kt = kernel_times(dade, torch, ix, Qd, w.k, npb, max(3, args.steps // 4), **kw)
        # algorithmic bytes of the DCO kernel: stored coordinates up to each DCO's exit, plus the
        # id read and the key written for each kept candidate
        alg_round = s_bytes * int(st[1]) + 12 * int(st[2])
        ids_np, d2_np = ids.cpu().numpy(), d2.cpu().numpy()
        ex = np.array([[np.sum((X[i].astype(np.float64) - Q[q]) ** 2) for i in ids_np[q]] for q in range(nq)])
        rel = np.abs(d2_np - ex) / np.maximum(ex, 1e-30)
        res[mode] = dict(nprobe=npb, p_s=ps_m, recall=r_m, qps=nq / (ms / 1e3), ms_per_step=ms,
                         p50_ms=float(np.percentile(walls, 50)), p99_ms=float(np.percentile(walls, 99)),
                         times=kt, dcos=int(st[0]), dims_frac=float(st[1]) / max(1, st[0] * w.dim),
                         kept=int(st[2]), reranked=int(st[3]), alg_round=alg_round, record=rec,
                         max_rel_err=float(rel.max()), mean_rel_err=float(rel.mean()))
        log(f"[bench] {mode}: nprobe {npb} recall {r_m:.4f} {res[mode]['qps']:.0f} QPS ({ms:.3f} ms/step) "
            f"round kernels {kt['round_kernel_ms']:.3f} ms over {kt['round_launches']:.0f} launches, "
            f"dims {res[mode]['dims_frac']:.4f}")

    d = res["dade"]
    kt = d["times"]
    launches = kt["round_launches"]
    avg_ms = kt["round_kernel_ms"] / launches
    achieved = d["alg_round"] / (kt["round_kernel_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profile(w.name, store, d["nprobe"], d["p_s"])
    traffic_gbs = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
    out = {
        "metric": METRIC, "value": round(d["qps"], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(d["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{store} store, f32 accumulate" if store != "f32" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "nlist": w.nlist, "k": w.k,
                   "queries_per_step": nq, "nprobe": d["nprobe"], "delta_d": w.delta_d, "p_s": d["p_s"],
                   "store": store, "schedule": SCHEDULE["schedule"], "fill_min": SCHEDULE["fill_min"],
                   "growth": SCHEDULE["growth"], "rerank_rule": args.rerank, f"recall@{w.k}": round(d["recall"], 4)},
        "search_record": d["record"],
        "p50_ms": round(d["p50_ms"], 4), "p99_ms": round(d["p99_ms"], 4),
        "full_d": {"qps": round(res["full_d"]["qps"], 1), "nprobe": res["full_d"]["nprobe"],
                   f"recall@{w.k}": round(res["full_d"]["recall"], 4),
                   "ms_per_step": round(res["full_d"]["ms_per_step"], 4),
                   "p50_ms": round(res["full_d"]["p50_ms"], 4), "p99_ms": round(res["full_d"]["p99_ms"], 4)},
        "speedup_vs_full_d": round(d["qps"] / res["full_d"]["qps"], 3),
        "comparison": "each method at its own fastest configuration reaching the recall target",
        "stages_ms": {k_: round(v, 4) for k_, v in kt.items()},
        "dims_read_frac": round(d["dims_frac"], 4),
        "reranked_per_query": round(d["reranked"] / nq, 2),
        "dist2_rel_err_vs_fp64": {"max": d["max_rel_err"], "mean": d["mean_rel_err"]},
        "recall_sweep": {"full_d": {str(k_): round(v, 4) for k_, v in sweep["full_d"].items()},
                         "dade_by_p_s": {ps_: {str(k_): round(v, 4) for k_, v in c.items()}
                                         for ps_, c in sweep["dade"].items()}},
        "roofline": {"bound": "hbm", "kernel": "scan_round_kernel", "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": (round(traffic_gbs, 1) if traffic else None),
                     "frac_counted": (round(traffic_gbs / PEAK_HBM_GBS, 4) if traffic else None),
                     "alg_bytes_per_launch": round(d["alg_round"] / launches), "launches_per_step": launches,
                     "avg_launch_ms": round(avg_ms, 5),
                     "limiter": "the HBM roof applies by arithmetic intensity (1 FLOP/B for a 16-bit store); the "
                                "kernel runs below it, limited by the latency of each round's deepest DCO chains; "
                                "counted DRAM bytes are below the algorithmic ones where lists are re-read from "
                                "L2 / Infinity Cache"},
    }
    if store != "f32":
        # the lazy rerank rule at the same operating point (fewer exact distances; it keeps what the
        # plain rule keeps unless a skipped candidate's stored-precision error exceeds delta)
        other = "lazy" if args.rerank == "all" else "all"
        kw = dict(delta_d=w.delta_d, rerank_rule=other, **SCHEDULE)
        stats = torch.zeros((nq, 4), dtype=torch.int64, device=dev)
        ids_o, _ = dade.dade_search(ix, Qd, w.k, d["nprobe"], stats=stats, **kw)
        torch.cuda.synchronize()
        ms = throughput(dade, torch, ix, Qd, w.k, d["nprobe"], args.steps, args.warmup, **kw)
        ids_main, _ = dade.dade_search(ix, Qd, w.k, d["nprobe"], delta_d=w.delta_d, **SCHEDULE, **RR)
        torch.cuda.synchronize()
        a_, b_ = ids_o.cpu().numpy(), ids_main.cpu().numpy()
        out["rerank_" + other] = {"qps": round(nq / (ms / 1e3), 1), f"recall@{w.k}": round(recall_at(a_, gt, w.k), 4),
                                  "reranked_per_query": round(float(stats[:, 3].sum().item()) / nq, 2),
                                  "queries_differing_from_" + args.rerank: int(sum(
                                      set(a_[i].tolist()) != set(b_[i].tolist()) for i in range(nq)))}
        log(f"[bench] rerank rule {other}: {out['rerank_' + other]}")
    if not args.no_serving:
        mib = args.serve_budget_mib or 512
        out["serving"] = serving_sweep(dade, ix, Q, gt, w.k, (w.k,), (d["nprobe"],), budget=mib << 20, seed=w.seed,
                                       delta_d=w.delta_d, **SCHEDULE)
    if not args.no_tune:
        # the autotuner at the operating point: agreement with FULL_D at this nprobe (whose recall is
        # 1.0 here) bounded by the recall target
        chosen, table = dade.dade_autotune(ix, Qd, w.k, d["nprobe"], min_agreement=args.target, reps=5)
        ms = throughput(dade, torch, ix, Qd, w.k, d["nprobe"], max(3, args.steps // 4), 1, **chosen)
        ids_t, _ = dade.dade_search(ix, Qd, w.k, d["nprobe"], **chosen)
        torch.cuda.synchronize()
        out["autotune"] = {"min_agreement_with_full_d": args.target, "chosen": chosen,
                           "qps": round(nq / (ms / 1e3), 1), "recall@10": round(recall_at(ids_t.cpu().numpy(), gt,
                                                                                          w.k), 4),
                           "table": [{k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in t.items()}
                                     for t in table]}
        log(f"[bench] autotune: {chosen} -> {out['autotune']['qps']:.0f} QPS, recall "
            f"{out['autotune']['recall@10']:.4f}")
    if not args.no_graph_study:
        out["graph"] = graph_study(dade, torch, args.target, max(3, args.steps // 4))
        out["graph_highd_sample"] = graph_study(dade, torch, args.target, max(3, args.steps // 4),
                                                sample=(w, X, Q, d["p_s"]))
    if not args.no_variants and store != "f32":
        # the same lists and transform with the other 16-bit store and with FP32 (recall vs FP32)
        art = dade.dade_export(ix)
        variants = {}
        ids_main, _ = dade.dade_search(ix, Qd, w.k, d["nprobe"], delta_d=w.delta_d, **SCHEDULE)
        for vs in ("f16" if store == "bf16" else "bf16", "f32"):
            vi = dade.dade_import({k_: v for k_, v in art.items() if k_ not in ("T",)}, Xd, store=vs)
            dade.dade_calibrate(vi, d["p_s"], pairs=pairs)
            ms = throughput(dade, torch, vi, Qd, w.k, d["nprobe"], max(3, args.steps // 4), 1,
                            delta_d=w.delta_d, **SCHEDULE)
            ids_v, d2_v = dade.dade_search(vi, Qd, w.k, d["nprobe"], delta_d=w.delta_d, **SCHEDULE)
            torch.cuda.synchronize()
            ids_v, d2_v = ids_v.cpu().numpy(), d2_v.cpu().numpy()
            ex = np.array([[np.sum((X[i].astype(np.float64) - Q[q]) ** 2) for i in ids_v[q]] for q in range(nq)])
            rel = np.abs(d2_v - ex) / np.maximum(ex, 1e-30)
            variants[vs] = {"qps": round(nq / (ms / 1e3), 1), "recall@10": round(recall_at(ids_v, gt, w.k), 4),
                            "dist2_rel_err_max": float(rel.max())}
            if vs == "f32":
                out["recall@10_vs_f32_path"] = round(recall_at(ids_main.cpu().numpy(), ids_v, w.k), 4)
            vi.close()
        out["variants"] = variants
    if not args.no_ablation:
        out["ablation"] = oblivious_ablation(dade, torch, ix, Xd, Qd, w, gt, store, pairs, d["nprobe"],
                                             max(3, args.steps // 4))
    if not args.no_linear:
        out["linear_scan"] = linear_scan(dade, torch, w, store, d["p_s"], max(3, args.steps // 4))
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        dade.dade_calibrate(ix, d["p_s"], pairs=pairs)   # the ablation leaves another P_s behind
        out["cpu_baseline"] = cpu_baseline(w, X, Q, dade.dade_export(ix), store, d["nprobe"], d["p_s"], args.rerank,
                                           gt, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
