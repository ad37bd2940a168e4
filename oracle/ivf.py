"""IVF search with DADE distance comparisons, in float64.

Follows the end of the Methodology section: IVF selects the N_probe clusters whose
centroids are nearest to the query, then scans their candidates while keeping the KNN set
in a max-heap of size K; each candidate gets one DCO against the heap's maximum distance
and, when the DCO answers yes, the heap is updated.  The DCO is Algorithm 1 with the
estimate of Eq. (13) and the test built on eps_d of Eq. (14) (see ``estimator``), or
FDScanning when ``mode="exact"``.

Readings where the paper is silent (each is a parameter or stated rule here):
* k-means lists (Experiments: Faiss k-means, N_c about sqrt(N)): Lloyd iterations from
  seed rows that are passed in; an empty cluster keeps its centroid; distance ties go to
  the lower centroid id; rows are finally assigned to the last centroids and each list
  holds its rows in ascending row id.
* Probe order: ascending (squared centroid distance, list id).
* Heap order: the total order on (squared distance, id).  r is the square root of the
  K-th smallest squared distance held, or +inf while fewer than K are held.  A candidate
  that survives every test is kept iff the heap is not full or (dist^2, id) < (r^2, id_r).
* Round schedule (fixes the threshold each DCO sees): the candidate sequence (probed lists
  concatenated in probe order) is split into rounds; every candidate of a round is compared
  against the heap as it was when the round started, and the round's accepted candidates
  are merged in at its end.  The first round is the first max(K, fill_min) candidates (they
  fill the heap); after it, ``per_rank`` ends a round at every list end, ``doubling`` at
  the ends of probe ranks 1, 2, 4, 8, ..., and ``whole`` only at the end of the sequence; a
  round is also cut once it holds growth times the candidates scanned before it
  (``round_starts``); ``sequential`` = one candidate
  per round in list order, i.e. the heap is updated after every DCO exactly as the paper
  describes.

Low-precision index (not in the paper): tests use the stored coordinates; a survivor whose
stored-precision S_D exceeds (1 + delta) r^2 is dropped (the gate).  Two rules then give the
survivors their exact distances: ``rerank="all"`` reranks every survivor that passed the gate
(the plain rule, the default); ``rerank="lazy"`` reranks the K smallest and the others only if
their stored-precision S_D is within (1 + delta) of the K-th exact distance known at that point
(``_rerank_lazy``).  The keep rule above then applies to the exact distances.

Near ties (for comparisons with a search computed in lower precision): with ``log=True`` every
decision whose relative margin is small -- a test, a gate, a keep compare, the cut between the
K-th and (K+1)-th key, a gap in the probe order -- is logged with a key naming it, and ``flips``
re-runs a query with chosen decisions taken the other way.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import estimator, pca


# ----------------------------------------------------------------------------- k-means

def _sqdist(A, B, chunk=16_384, direct_limit=100_000_000):
    """Exact float64 squared distances between rows of A and rows of B ([len(A), len(B)])."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape[0] * B.shape[0] * A.shape[1] <= direct_limit:
        return np.stack([np.sum((B - a) ** 2, axis=1) for a in A]) if len(A) else np.zeros((0, len(B)))
    out = np.empty((A.shape[0], B.shape[0]))
    bn = np.einsum("ij,ij->i", B, B)
    for s in range(0, A.shape[0], chunk):
        a = A[s:s + chunk]
        an = np.einsum("ij,ij->i", a, a)
        out[s:s + chunk] = np.maximum(an[:, None] - 2.0 * (a @ B.T) + bn[None, :], 0.0)
    return out


def assign(X, C, chunk=65_536) -> np.ndarray:
    """Nearest centroid per row; ties to the lower centroid id (argmin keeps the first)."""
    X = np.asarray(X)
    lab = np.empty(X.shape[0], dtype=np.int64)
    for s in range(0, X.shape[0], chunk):
        lab[s:s + chunk] = np.argmin(_sqdist(X[s:s + chunk], C), axis=1)
    return lab


def kmeans(X, init_rows, iters: int = 10) -> np.ndarray:
    """Lloyd's algorithm from the seed rows ``init_rows``; returns float64 centroids."""
    X = np.asarray(X)
    C = X[np.asarray(init_rows)].astype(np.float64)
    for _ in range(iters):
        lab = assign(X, C)
        counts = np.bincount(lab, minlength=C.shape[0])
        order = np.argsort(lab, kind="stable")
        nonempty = np.nonzero(counts)[0]
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])[nonempty]
        sums = np.add.reduceat(X[order].astype(np.float64), starts, axis=0)
        C[nonempty] = sums / counts[nonempty, None]
    return C


def objective(X, C, lab) -> float:
    """Mean squared distance of each row to its assigned centroid."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.mean(np.sum((X - np.asarray(C)[lab]) ** 2, axis=1)))


def build_lists(lab, nlist: int):
    """(offsets [nlist+1], ids [N]): rows grouped by list, ascending row id inside a list."""
    order = np.argsort(np.asarray(lab), kind="stable").astype(np.int64)
    counts = np.bincount(lab, minlength=nlist)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64), order


def probe_order(q_rot, cent_rot, nprobe: int):
    """(list ids, squared distances) of the nprobe nearest centroids, by (dist^2, list id)."""
    d2 = np.sum((np.asarray(cent_rot, dtype=np.float64) - q_rot) ** 2, axis=1)
    order = np.lexsort((np.arange(len(d2)), d2))
    return order[:nprobe], d2[order]


# ----------------------------------------------------------------------------- index

@dataclasses.dataclass
class Index:
    """Everything a search reads.  ``Y[ids]`` returns the stored rotated rows (float64)."""
    mu: np.ndarray
    W: np.ndarray
    lam: np.ndarray
    eps: np.ndarray            # eps_d, d = 1..D (Eq. (14))
    centroids: np.ndarray      # original basis
    offsets: np.ndarray
    ids: np.ndarray
    Y: object                  # stored rotated coordinates, indexable by row id
    Y_exact: object = None     # exact rotated coordinates for the low-precision rerank
    delta: float = 0.0         # rerank margin
    T: np.ndarray = None       # reduced-form thresholds T_d (same decisions as eps_d)

    @property
    def dim(self):
        return self.W.shape[0]

    @property
    def nlist(self):
        return len(self.offsets) - 1

    def cent_rot(self):
        return pca.rotate(self.centroids, self.mu, self.W)


class LazyRotated:
    """Rotated rows computed on demand: rows -> (X[rows] - mu) @ W (optionally rounded)."""

    def __init__(self, X, mu, W, rounding=None):
        self.X, self.mu, self.W, self.rounding = X, mu, W, rounding

    def __getitem__(self, rows):
        y = pca.rotate(np.asarray(self.X)[rows], self.mu, self.W)
        return self.rounding(y) if self.rounding is not None else y


def build(X, nlist, init_rows, pairs, p_s=0.1, iters=10, store=None, rotation=None):
    """Oracle index: transform, k-means lists and eps_d from the given pairs.

    ``store`` (callable on rotated rows, e.g. ``lowp`` rounding) makes a low-precision
    index: tests read the rounded coordinates, eps_d and delta are calibrated on them.
    ``rotation`` (an orthogonal D x D matrix, columns the axes) replaces the data-aware W: the
    data-oblivious comparison of Figure 1, with lambda_k the variance along each axis and the
    same empirical calibration of eps_d.
    """
    from . import lowp
    mu, W, lam = pca.fit(X)
    if rotation is not None:
        W = np.asarray(rotation, dtype=np.float64)
        lam = pca.axis_variances(X, mu, W)
    C = kmeans(X, init_rows, iters)
    offsets, ids = build_lists(assign(X, C), nlist)
    Y = pca.rotate(X, mu, W)
    if store is None:
        eps, T, _ = estimator.calibrate(X, W, lam, pairs, p_s)
        return Index(mu, W, lam, eps, C, offsets, ids, Y, T=T)
    Ys = store(Y)
    eps, T, _ = estimator.calibrate(X, W, lam, pairs, p_s, stored=Ys)
    delta = lowp.rerank_margin(X, pairs, Ys)
    return Index(mu, W, lam, eps, C, offsets, ids, Ys, Y_exact=Y, delta=delta, T=T)


# ----------------------------------------------------------------------------- search

def round_bounds(nprobe: int, schedule: str):
    """Probe-rank ranges [lo, hi) of each round."""
    if schedule == "per_rank":
        return [(t, t + 1) for t in range(nprobe)]
    if schedule == "doubling":
        b, x = [0], 1
        while x < nprobe:
            b.append(x)
            x *= 2
        b.append(nprobe)
        return list(zip(b[:-1], b[1:]))
    if schedule == "whole":   # the probe ranks form one range: no cut at a list end
        return [(0, nprobe)]
    raise ValueError(schedule)


# Round-size defaults shared with the GPU path's search options (they are part of what a
# search computes, so both sides take them as parameters).
FILL_MIN = 32   # the first round holds at least this many candidates
GROWTH = 16     # a later round holds at most GROWTH times the candidates before it


def round_starts(sizes, K: int, schedule: str, fill_min: int = FILL_MIN, growth: int = GROWTH) -> list:
    """Round boundaries in the candidate sequence (probed lists concatenated in probe order).

    The first round holds the first max(K, fill_min) candidates: they fill the heap, as the
    paper's IVF fills its max-heap before any comparison can fail (a larger first round gives
    the following rounds a tighter r).  A later round that starts after s candidates ends at the
    first schedule cut after s (``round_bounds``: where the schedule's probe ranks end) or after
    growth * s candidates if that comes first (growth = 0: no such cap).  Returns the positions
    0 = b_0 < b_1 < ... = total.
    """
    ends = np.cumsum(sizes)
    total = int(ends[-1]) if len(ends) else 0
    pos = min(max(K, fill_min), total)
    cuts = sorted(set([int(ends[hi - 1]) for _, hi in round_bounds(len(sizes), schedule)] + [total]))
    out = [0] + ([pos] if pos > 0 else [])
    while pos < total:
        nxt = min(c for c in cuts if c > pos)
        if growth > 0:
            nxt = min(nxt, pos + growth * pos)
        out.append(nxt)
        pos = nxt
    return out


def tested_dims(D: int, delta_d: int) -> np.ndarray:
    """d = Delta_d, 2 Delta_d, ... strictly below D (Algorithm 1 with the d <= D reading)."""
    return np.arange(delta_d, D, delta_d, dtype=np.int64)


def _flipped(flips, kind, rnd):
    """Keys of the decisions of one kind in round ``rnd`` that a re-run takes the other way."""
    return [k for k in flips if k[0] == kind and k[1] == rnd]


def _note(events, tol, rel, key):
    """Record a decision whose relative margin is at most ``tol`` (a near tie)."""
    if events is not None and rel <= tol:
        events.append((float(rel), key))


def _merge(hd, hi, d2, ids, K, rnd=0, flips=(), events=None, tol=0.0):
    """The K smallest (dist^2, id) of the heap and the round's kept candidates.

    The decision at the cut (which of the K-th and (K+1)-th keys stays) is a near tie when
    their distances differ by little; ``("cut", round, id_K, id_K+1)`` in ``flips`` keeps the
    (K+1)-th instead.  Returns (dist^2, ids, relative gap at the cut).
    """
    d = np.concatenate([hd, d2])
    i = np.concatenate([hi, ids])
    o = np.lexsort((i, d))
    gap = math.inf
    if len(o) > K:
        key = ("cut", rnd, int(i[o[K - 1]]), int(i[o[K]]))
        if d[o[K - 1]] > 0:
            gap = abs(d[o[K]] - d[o[K - 1]]) / d[o[K - 1]]
        elif d[o[K]] == 0:
            gap = 0.0
        _note(events, tol, gap, key)
        if key in flips:
            o = o.copy()
            o[K - 1], o[K] = o[K], o[K - 1]
    return d[o[:K]], i[o[:K]], gap


def _gate(index, cand, SD, alive, full, r2, rnd, flips, events, tol):
    """The low-precision gate: a survivor goes on to the exact rerank when the heap is not
    full or its stored-precision S_D <= (1 + delta) r^2.  Returns (mask, smallest margin)."""
    A = alive.copy()
    margin = math.inf
    if full:
        gate = (1.0 + index.delta) * r2
        ok = SD <= gate
        for k in _flipped(flips, "gate", rnd):
            ok[cand == k[2]] = ~ok[cand == k[2]]
        for j in np.nonzero(alive)[0]:
            rel = abs(SD[j] - gate) / gate if gate > 0 else math.inf
            margin = min(margin, rel)
            _note(events, tol, rel, ("gate", rnd, int(cand[j])))
        A &= ok
    return A, margin


def _exact(index, q, cand, mask, SD):
    """Stored-precision S_D replaced by the exact squared distance where ``mask`` is set."""
    exact = SD.copy()
    if mask.any():
        dx = index.Y_exact[cand[mask]] - q
        exact[mask] = np.sum(dx * dx, axis=1)
    return exact


def _rerank_all(index, q, cand, SD, alive, full, r2, rnd=0, flips=(), events=None, tol=0.0):
    """Low-precision rerank, plain rule: every survivor that passes the gate gets its exact
    squared distance.  Returns the reranked mask, the distances to keep-test and the smallest
    relative margin of the gates."""
    A, margin = _gate(index, cand, SD, alive, full, r2, rnd, flips, events, tol)
    return A, _exact(index, q, cand, A, SD), margin


def _rerank_lazy(index, q, cand, SD, alive, full, r2, hd, hi, K, rnd=0, flips=(), events=None, tol=0.0):
    """Low-precision rerank, lazy rule (fewer exact distances than the plain rule).

    A = survivors that pass the gate.  F = the K smallest of A by (S_D, id); they are reranked
    exactly.  b = the K-th smallest exact distance of the heap and F (+inf if fewer than K);
    the rest of A is reranked only where S_D <= (1 + delta) b.  When no candidate it skips has
    a stored-precision error above delta, the round keeps what the plain rule keeps (a
    skipped candidate's exact distance then exceeds b, which bounds the round's K-th).
    Decision keys for re-runs: ``("gate", round, id)``, ``("fsel", round, id_K, id_K+1)`` (the
    cut between F and the rest) and ``("bound", round, id)``.
    """
    delta = index.delta
    A, margin = _gate(index, cand, SD, alive, full, r2, rnd, flips, events, tol)
    ia = np.nonzero(A)[0]
    o = ia[np.lexsort((cand[ia], SD[ia]))]
    if len(o) > K:
        key = ("fsel", rnd, int(cand[o[K - 1]]), int(cand[o[K]]))
        if SD[o[K - 1]] > 0:
            rel = abs(SD[o[K]] - SD[o[K - 1]]) / SD[o[K - 1]]
            margin = min(margin, rel)
            _note(events, tol, rel, key)
        if key in flips:
            o = o.copy()
            o[K - 1], o[K] = o[K], o[K - 1]
    F, rest = o[:K], o[K:]
    mF = np.zeros_like(alive)
    mF[F] = True
    exact = _exact(index, q, cand, mF, SD)
    pool_d = np.concatenate([hd, exact[F]])
    pool_i = np.concatenate([hi, cand[F]])
    b = math.inf
    if len(pool_d) >= K:
        b = float(pool_d[np.lexsort((pool_i, pool_d))[K - 1]])
    bound = (1.0 + delta) * b
    inside = SD[rest] <= bound
    for k in _flipped(flips, "bound", rnd):
        inside[cand[rest] == k[2]] = ~inside[cand[rest] == k[2]]
    if math.isfinite(bound) and bound > 0:
        for j in rest:
            rel = abs(SD[j] - bound) / bound
            margin = min(margin, rel)
            _note(events, tol, rel, ("bound", rnd, int(cand[j])))
    R = mF.copy()
    R[rest[inside]] = True
    return R, _exact(index, q, cand, R, exact), margin


# Low-precision rerank rules (the paper has no low-precision store; see the module header).
RERANK_RULES = ("all", "lazy")


def _scan_round(index, q, cand, hd, hi, K, delta_d, mode, tests, rerank="all", rnd=0, flips=(),
                events=None, tol=0.0):
    """DCOs of one round against the snapshot heap (hd, hi).  Returns accepted + logs.

    ``flips`` holds decision keys to take the other way (a re-run that explains a result
    computed in lower precision): ``("test", round, id, d)`` for the test of candidate ``id``
    at dimension d, ``("keep", round, id)`` for its keep compare, and the rerank keys.
    Decisions within relative margin ``tol`` are appended to ``events`` as (margin, key).
    """
    D = index.dim
    full = len(hd) == K
    r2 = float(hd[-1]) if full else math.inf
    idr = int(hi[-1]) if full else -1
    r = math.sqrt(r2)
    diff = index.Y[cand] - q
    S = np.cumsum(diff * diff, axis=1)
    n = len(cand)
    margin = math.inf
    exit_d = np.full(n, D, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    if mode == "dade" and len(tests) and full:
        c = estimator.scale(index.lam)
        est = estimator.estimate(S[:, tests - 1], c[tests - 1][None, :])
        rej = estimator.reject(est, index.eps[tests - 1][None, :], r)
        for k in _flipped(flips, "test", rnd):
            rows, cols = np.nonzero(cand == k[2])[0], np.nonzero(tests == k[3])[0]
            for i in rows:
                rej[i, cols] = ~rej[i, cols]
        anyrej = rej.any(axis=1)
        first = np.where(anyrej, rej.argmax(axis=1), len(tests) - 1)
        exit_d = np.where(anyrej, tests[first], D)
        alive = ~anyrej
        bound2 = ((1.0 + index.eps[tests - 1]) * r) ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.abs(est ** 2 - bound2[None, :]) / bound2[None, :]
        seen = np.arange(len(tests))[None, :] <= np.where(anyrej, first, len(tests) - 1)[:, None]
        rel = np.where(seen & np.isfinite(rel), rel, math.inf)
        if rel.size:
            margin = min(margin, float(rel.min()))
        if events is not None:
            for i, j in zip(*np.nonzero(rel <= tol)):
                events.append((float(rel[i, j]), ("test", rnd, int(cand[i]), int(tests[j]))))
    SD = S[:, -1]
    if index.Y_exact is not None:
        if rerank == "all":
            alive, SD, m2 = _rerank_all(index, q, cand, SD, alive, full, r2, rnd, flips, events, tol)
        elif rerank == "lazy":
            alive, SD, m2 = _rerank_lazy(index, q, cand, SD, alive, full, r2, hd, hi, K, rnd, flips, events, tol)
        else:
            raise ValueError(rerank)
        margin = min(margin, m2)
    if full:
        below = (SD < r2) | ((SD == r2) & (cand < idr))
        for k in _flipped(flips, "keep", rnd):
            below[cand == k[2]] = ~below[cand == k[2]]
        keep = alive & below
        if r2 > 0:
            for j in np.nonzero(alive)[0]:
                rel = abs(SD[j] - r2) / r2
                margin = min(margin, rel)
                _note(events, tol, rel, ("keep", rnd, int(cand[j])))
    else:
        keep = alive
    return SD[keep], cand[keep], exit_d, margin, int(alive.sum())


def search(index: Index, Q, K, nprobe, delta_d: int, mode: str = "dade",
           schedule: str = "per_rank", log: bool = False, q_rot=None,
           fill_min: int = FILL_MIN, growth: int = GROWTH, rerank: str = "all", flips=None,
           event_tol: float = 1e-3):
    """IVF search.  K and nprobe are ints or per-query arrays; rounds follow ``round_starts``.

    Returns (ids [nq, Kmax] int64 with -1 padding, dist2 [nq, Kmax] with +inf padding, logs).
    ``logs`` (when requested) holds per-query: dcos, dims (sum of d_exit), accepted,
    survivors (reached d = D), rounds, min_margin (smallest relative margin of any test,
    rerank gate, keep compare or top-K cut), probe_gap (smallest relative gap between
    consecutive probe-order distances, up to the first list not probed) and ``events``: a list
    per query of (relative margin, decision key) for every decision within ``event_tol``.
    ``rerank`` picks the low-precision rerank rule ("all" or "lazy"); ``flips`` maps a query
    index to decision keys taken the other way (``("probe", t)`` swaps probe ranks t, t+1).
    """
    Q = np.asarray(Q)
    nq = Q.shape[0]
    flips = flips or {}
    Ks = np.broadcast_to(np.asarray(K, dtype=np.int64), (nq,))
    nps = np.minimum(np.broadcast_to(np.asarray(nprobe, dtype=np.int64), (nq,)), index.nlist)
    Kmax = int(Ks.max()) if nq else 0
    Qr = pca.rotate(Q, index.mu, index.W) if q_rot is None else np.asarray(q_rot, np.float64)
    cent = index.cent_rot()
    D = index.dim
    tests = tested_dims(D, delta_d)
    out_i = np.full((nq, Kmax), -1, dtype=np.int64)
    out_d = np.full((nq, Kmax), np.inf)
    logs = {k: np.zeros(nq, dtype=np.float64) for k in
            ("dcos", "dims", "accepted", "survivors", "rounds", "min_margin", "probe_gap")}
    logs["events"] = [[] for _ in range(nq)]
    for qi in range(nq):
        q = Qr[qi]
        fq = flips.get(qi, ())
        ev = logs["events"][qi]
        Kq, npq = int(Ks[qi]), int(nps[qi])
        order, d2c = probe_order(q, cent, index.nlist)
        order = order.copy()
        pg = math.inf
        for t in range(min(npq, index.nlist - 1)):   # gaps up to the first list not probed
            a, b = d2c[t], d2c[t + 1]
            rel = (b - a) / b if b > 0 else math.inf
            pg = min(pg, rel)
            _note(ev, event_tol, rel, ("probe", t))
        for k in fq:
            if k[0] == "probe":
                order[k[1]], order[k[1] + 1] = order[k[1] + 1], order[k[1]]
        logs["probe_gap"][qi] = pg
        probes = order[:npq]
        lists = [index.ids[index.offsets[l]:index.offsets[l + 1]] for l in probes]
        seq = np.concatenate(lists) if lists else np.zeros(0, np.int64)
        if schedule == "sequential":
            rounds = [seq[i:i + 1] for i in range(len(seq))]
        else:
            b = round_starts(np.array([len(x) for x in lists]), Kq, schedule, fill_min, growth)
            rounds = [seq[b0:b1] for b0, b1 in zip(b[:-1], b[1:])]
        hd = np.zeros(0)
        hi = np.zeros(0, dtype=np.int64)
        mm = math.inf
        for ri, cand in enumerate(rounds):
            logs["rounds"][qi] += 1
            if len(cand) == 0:
                continue
            d2, ids, exit_d, margin, surv = _scan_round(index, q, cand, hd, hi, Kq, delta_d, mode, tests,
                                                        rerank, ri, fq, ev, event_tol)
            logs["dcos"][qi] += len(cand)
            logs["dims"][qi] += float(exit_d.sum())
            logs["accepted"][qi] += len(ids)
            logs["survivors"][qi] += surv
            mm = min(mm, margin)
            hd, hi, gap = _merge(hd, hi, d2, ids, Kq, ri, fq, ev, event_tol)
            mm = min(mm, gap)
        logs["min_margin"][qi] = mm
        ev.sort(key=lambda e: e[0])
        out_i[qi, :len(hi)] = hi
        out_d[qi, :len(hd)] = hd
    return (out_i, out_d, logs) if log else (out_i, out_d)


def search_scalar(index: Index, Q, K: int, nprobe: int, delta_d: int, mode: str = "dade",
                  log: bool = False):
    """The paper's semantics, one candidate at a time: Algorithm 1 (or FDScanning) per
    candidate against the live heap maximum, heap updated after every DCO.

    A separate, scalar code path (``dco`` + an explicit heap) for small inputs; it must
    agree with ``search(..., schedule="sequential")``.
    """
    import heapq

    from . import dco
    Q = np.asarray(Q)
    Qr = pca.rotate(Q, index.mu, index.W)
    cent = index.cent_rot()
    c = estimator.scale(index.lam)
    out_i = np.full((len(Q), K), -1, dtype=np.int64)
    out_d = np.full((len(Q), K), np.inf)
    logs = {"dims": np.zeros(len(Q)), "accepted": np.zeros(len(Q))}
    for qi, q in enumerate(Qr):
        probes, _ = probe_order(q, cent, min(nprobe, index.nlist))
        heap = []  # entries (-dist2, -id): the root is the largest (dist2, id)
        for l in probes:
            for cid in index.ids[index.offsets[l]:index.offsets[l + 1]]:
                full = len(heap) == K
                r2 = -heap[0][0] if full else math.inf
                idr = -heap[0][1] if full else -1
                o = index.Y[np.array([cid])][0]
                if mode == "dade":
                    ok, dis, d_exit = dco.dade_dco(o, q, math.sqrt(r2), delta_d, index.eps, c)
                else:
                    ok, dis, d_exit = dco.fd_dco(o, q, math.sqrt(r2))
                logs["dims"][qi] += d_exit
                if not ok:
                    continue
                d2 = float(np.sum((q - o) ** 2))
                if full and not (d2 < r2 or (d2 == r2 and cid < idr)):
                    continue
                logs["accepted"][qi] += 1
                heapq.heappush(heap, (-d2, -int(cid)))
                if len(heap) > K:
                    heapq.heappop(heap)
        items = sorted((-a, -b) for a, b in heap)
        for j, (d2, cid) in enumerate(items):
            out_i[qi, j] = cid
            out_d[qi, j] = d2
    return (out_i, out_d, logs) if log else (out_i, out_d)
