"""Graph search with DADE distance comparisons, in float64 (test infrastructure only).

The paper's graph setting (HNSW** in the Experiments section) scans the neighbours of visited
objects, giving each one DCO against the maximum distance of the result set (size ef), and
discards a neighbour whose DCO answers no.  This oracle follows that search on a flat graph:

* Graph (reading; the paper uses HNSW's hierarchy, this oracle uses one layer and lets the
  entry points of the IVF lists play the part of the upper layers): every object's candidates
  are its nearest other objects by the index's exact IVF search (FDScanning over ``nprobe``
  lists), ordered by (dist^2, id), the object itself removed.  Its out-neighbours are the first
  ``degree`` of them, or, with ``candidates`` > 0, the ones HNSW's neighbour-selection heuristic
  keeps among the first ``candidates`` (``select_neighbors``); -1 padded; then up to
  ``reverse`` back links (``add_reverse_edges``).
* Entry points (reading): each IVF list's medoid (the member nearest its centroid, ties to the
  lower id) and the member farthest from the medoid (``list_entries``); a query starts from the
  entry points of its ``n_entry`` nearest lists (probe order).
* Beam: a pool of at most ``ef`` (dist^2, id) entries, each marked expanded or not.  Seeds enter
  with their full-D distance.  Each step expands the first unexpanded entry of the pool in
  (dist^2, id) order: its unvisited neighbours are marked visited and each gets one DCO (Algorithm
  1 at the given Delta_d, or FDScanning) against the pool's snapshot at the step's start
  (r^2 = the ef-th distance, +inf while the pool holds fewer than ef), with the keep rule of the
  IVF oracle; the kept ones are merged in (the ef smallest stay).  The search stops when every
  pool entry is expanded or after ``max_iters`` expansions.
* Low-precision stores: DCOs and the pool use the stored coordinates; at the end every pool
  entry is reranked with the exact coordinates and the K smallest by (exact dist^2, id) are
  returned.  With an FP32 store the final distances are the stored ones recomputed exactly.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import ivf, pca


def build_knn_graph(index: ivf.Index, X, degree: int, nprobe: int, delta_d: int = 32, rows=None,
                    candidates: int = 0, log: bool = False):
    """[len(rows) x degree] int64 out-neighbours (row ids, -1 padded) of the given rows (all rows
    by default) from the index's FDScanning search: the ``degree`` nearest other rows, or with
    ``candidates`` > 0 the ones ``select_neighbors`` keeps among the ``candidates`` nearest.
    With ``log``, also a dict of per-row margins: ``boundary``, the relative gap between the last
    candidate taken and the next one (a near tie there can swap the candidate set), and
    ``select``, the heuristic's smallest decision margin (inf without selection)."""
    X = np.asarray(X)
    rows = np.arange(len(X)) if rows is None else np.asarray(rows)
    take = candidates if candidates > 0 else degree
    ids, d2 = ivf.search(index, X[rows], take + 2, nprobe, delta_d, mode="full_d", schedule="doubling")[:2]
    out = np.full((len(rows), degree), -1, dtype=np.int64)
    info = {"boundary": np.full(len(rows), np.inf), "select": np.full(len(rows), np.inf)}
    for i, r in enumerate(rows):
        keep = [j for j in range(take + 2) if ids[i, j] >= 0 and ids[i, j] != r]
        row = [int(ids[i, j]) for j in keep[:take]]
        if len(keep) > take and d2[i, keep[take - 1]] > 0:
            a, b = d2[i, keep[take - 1]], d2[i, keep[take]]
            info["boundary"][i] = abs(b - a) / a
        if candidates > 0:
            row, info["select"][i] = select_neighbors(X, int(r), row, degree)
        out[i, :len(row)] = row[:degree]
    return (out, info) if log else out


def select_neighbors(X, v: int, cands, M: int):
    """HNSW's neighbour-selection heuristic (Malkov and Yashunin, the simple form: no candidate
    extension, pruned candidates not added back) for object v, in float64 over the rows of X.

    Candidates are taken in ascending (dist^2 to v, id) order.  A candidate e is pruned when some
    neighbour already kept is strictly closer to e than v is (d(e, r) < d(e, v)), and kept
    otherwise, until M are kept.  Returns (kept ids in the order kept, margin): margin is the
    smallest relative gap among the quantities the decisions compare, |d(e, r) - d(e, v)| over
    d(e, v) for the nearest kept r of every candidate examined, and the gaps between consecutive
    candidate distances (their order)."""
    X = np.asarray(X, dtype=np.float64)
    cands = np.asarray([int(c) for c in cands if c >= 0 and c != v], dtype=np.int64)
    if len(cands) == 0 or M < 1:
        return [], np.inf
    dv = np.sum((X[cands] - X[v]) ** 2, axis=1)
    order = np.lexsort((cands, dv))
    cands, dv = cands[order], dv[order]
    margin = np.inf
    if len(dv) > 1:
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.abs(np.diff(dv)) / np.maximum(dv[1:], 1e-300)
        margin = float(g.min())
    kept = []
    for e, de in zip(cands, dv):
        if len(kept) == M:
            break
        if kept:
            dr = np.sum((X[kept] - X[e]) ** 2, axis=1).min()
            margin = min(margin, abs(dr - de) / max(de, 1e-300))
            if dr < de:
                continue
        kept.append(int(e))
    return kept, margin


def add_reverse_edges(neighbors, X, reverse: int) -> np.ndarray:
    """Rows of degree + reverse: each row's out-neighbours, then up to `reverse` of the rows that
    list it as an out-neighbour and it does not list already, nearest first by (dist^2, id);
    -1 padded (reading: one-layer graphs are made navigable by linking back, as HNSW's
    bidirectional links do)."""
    neighbors = np.asarray(neighbors)
    n, deg = neighbors.shape
    X = np.asarray(X, dtype=np.float64)
    incoming = [[] for _ in range(n)]
    for u in range(n):
        for v in neighbors[u]:
            if v >= 0:
                incoming[int(v)].append(u)
    out = np.full((n, deg + reverse), -1, dtype=np.int64)
    for v in range(n):
        fwd = [int(u) for u in neighbors[v] if u >= 0]
        out[v, :len(fwd)] = fwd
        cand = np.array(sorted(set(incoming[v]) - set(fwd)), dtype=np.int64)
        if reverse == 0 or len(cand) == 0:
            continue
        d2 = np.sum((X[cand] - X[v]) ** 2, axis=1)
        chosen = cand[np.lexsort((cand, d2))[:reverse]]
        out[v, len(fwd):len(fwd) + len(chosen)] = chosen
    return out


def list_entries(index: ivf.Index, X) -> np.ndarray:
    """[nlist x 2] row ids: each list's medoid, then the member farthest from the medoid (ties to
    the lower id; -1 when the list has fewer than two members).  A two-point farthest-first cover
    of the list (reading): a k-means list that spans two mixture components gets an entry in
    each, and a kNN graph has no edges between components."""
    X = np.asarray(X, dtype=np.float64)
    med = list_medoids(index, X)
    out = np.full((index.nlist, 2), -1, dtype=np.int64)
    out[:, 0] = med
    for l in range(index.nlist):
        members = index.ids[index.offsets[l]:index.offsets[l + 1]]
        if len(members) < 2:
            continue
        d2 = np.sum((X[members] - X[med[l]]) ** 2, axis=1)
        out[l, 1] = members[np.lexsort((members, -d2))[0]]
    return out


def list_medoids(index: ivf.Index, X) -> np.ndarray:
    """[nlist] row id of each list's member nearest its centroid (ties: lower id), -1 if empty."""
    X = np.asarray(X, dtype=np.float64)
    out = np.full(index.nlist, -1, dtype=np.int64)
    for l in range(index.nlist):
        members = index.ids[index.offsets[l]:index.offsets[l + 1]]
        if len(members) == 0:
            continue
        d2 = np.sum((X[members] - index.centroids[l]) ** 2, axis=1)
        out[l] = members[np.lexsort((members, d2))[0]]
    return out


def search(index: ivf.Index, neighbors, entries, Q, K: int, ef: int, n_entry: int, delta_d: int,
           mode: str = "dade", max_iters: int = 0, log: bool = False, flips=None, event_tol: float = 1e-3):
    """Beam search per query.  Returns (ids [nq, K] int64 -1 padded, dist2 [nq, K] +inf padded,
    logs) with logs per query: dcos, dims (sum of exit d), expansions, visited (count and, in
    visited_ids, the ids), min_margin (the smallest relative margin of any test, keep compare or
    merge boundary), probe_gap (the smallest relative gap between consecutive centroid
    distances up to the first list past the entry lists) and events (decisions within
    ``event_tol``, keyed as in ``ivf.search``: the seeds' merge is round 0, expansion s is round
    s, the final cut is round -1).  ``flips`` maps a query index to decision keys taken the
    other way."""
    Q = np.asarray(Q)
    nq = len(Q)
    max_iters = max_iters or 2 * ef
    beam = dataclasses.replace(index, Y_exact=None)   # DCOs and the pool on the stored coordinates
    exact_rows = index.Y_exact if index.Y_exact is not None else index.Y
    Qr = pca.rotate(Q, index.mu, index.W)
    cent = index.cent_rot()
    D = index.dim
    tests = ivf.tested_dims(D, delta_d)
    out_i = np.full((nq, K), -1, dtype=np.int64)
    out_d = np.full((nq, K), np.inf)
    logs = {k: np.zeros(nq) for k in ("dcos", "dims", "expansions", "visited")}
    logs["min_margin"] = np.full(nq, np.inf)
    logs["probe_gap"] = np.full(nq, np.inf)
    logs["visited_ids"] = []
    logs["events"] = [[] for _ in range(nq)]
    flips = flips or {}
    for qi in range(nq):
        q = Qr[qi]
        fq = flips.get(qi, ())
        ev = logs["events"][qi]
        ne = min(n_entry, index.nlist)
        order, cd = ivf.probe_order(q, cent, index.nlist)
        order = order.copy()
        head = cd[:ne + 1]   # the entry lists and the next one: a near tie can swap an entry list
        if len(head) > 1:
            with np.errstate(divide="ignore", invalid="ignore"):
                g = np.abs(np.diff(head)) / np.maximum(head[1:], 1e-300)
            logs["probe_gap"][qi] = float(g.min())
            for t, rel in enumerate(g):
                ivf._note(ev, event_tol, rel, ("probe", t))
        for k in fq:
            if k[0] == "probe":
                order[k[1]], order[k[1] + 1] = order[k[1] + 1], order[k[1]]
        lists = order[:ne]
        ent = np.asarray(entries).reshape(index.nlist, -1)   # one or two entry points per list
        seeds = np.array([int(e) for l in lists for e in ent[l] if e >= 0], dtype=np.int64)
        visited = set(seeds.tolist())
        diff = index.Y[seeds] - q
        sd = np.sum(diff * diff, axis=1)
        hd, hi, gap = ivf._merge(np.zeros(0), np.zeros(0, dtype=np.int64), sd, seeds, ef, 0, fq, ev, event_tol)
        margin = gap
        expanded = set()
        it = 0
        while it < max_iters:
            todo = [j for j in range(len(hi)) if int(hi[j]) not in expanded]
            if not todo:
                break
            c = int(hi[todo[0]])
            expanded.add(c)
            it += 1
            cand = np.array([u for u in neighbors[c] if u >= 0 and int(u) not in visited], dtype=np.int64)
            if len(cand) == 0:
                continue
            visited.update(cand.tolist())
            d2, ids, exit_d, m, _ = ivf._scan_round(beam, q, cand, hd, hi, ef, delta_d, mode, tests,
                                                    rnd=it, flips=fq, events=ev, tol=event_tol)
            logs["dcos"][qi] += len(cand)
            logs["dims"][qi] += exit_d.sum()
            hd, hi, gap = ivf._merge(hd, hi, d2, ids, ef, it, fq, ev, event_tol)
            margin = min(margin, m, gap)
        logs["expansions"][qi] = it
        logs["visited"][qi] = len(visited)
        logs["visited_ids"].append(np.array(sorted(visited), dtype=np.int64))
        # final pool: exact distances, the K smallest by (dist^2, id)
        de = exact_rows[hi] - q
        ex = np.sum(de * de, axis=1)
        o = np.lexsort((hi, ex))
        if len(o) > K and ex[o[K - 1]] > 0:
            rel = abs(ex[o[K]] - ex[o[K - 1]]) / ex[o[K - 1]]
            margin = min(margin, rel)
            key = ("cut", -1, int(hi[o[K - 1]]), int(hi[o[K]]))
            ivf._note(ev, event_tol, rel, key)
            if key in fq:
                o = o.copy()
                o[K - 1], o[K] = o[K], o[K - 1]
        o = o[:K]
        ev.sort(key=lambda e: e[0])
        out_i[qi, :len(o)] = hi[o]
        out_d[qi, :len(o)] = ex[o]
        logs["min_margin"][qi] = margin
    return out_i, out_d, (logs if log else None)
