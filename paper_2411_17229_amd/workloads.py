"""Seeded synthetic workloads shaped like the paper's datasets (Experiments, Table 1).

This module only draws random inputs: base vectors, queries, k-means seed rows,
calibration pairs, per-query (K, nprobe) and request arrivals.  It holds none of
DADE's arithmetic, so both the HIP path and the FP64 oracle can be fed from it.

Generator (one seed, independent streams spawned from ``numpy.random.SeedSequence``):
  * C mixture centres m_c ~ N(0, 4 I)  (standard deviation 2);
  * one Haar-random rotation R shared by every component (QR of a Gaussian
    matrix, column signs fixed by the signs of diag(R_qr));
  * per-component spectrum lam_i = s * i**(-beta), i = 1..D, with s chosen so
    that the mean of lam is 1;
  * x = m_c + R (sqrt(lam) * z), z ~ N(0, I), c uniform over components;
  * queries are drawn from the same mixture on their own streams.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAMS = ("centres", "rotation", "labels", "noise", "q_labels", "q_noise",
           "kmeans_init", "calib_pairs", "batch_params", "arrivals")


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload.  Sizes follow the paper's Table 1 shapes."""
    name: str
    n: int
    dim: int
    components: int
    beta: float
    n_queries: int
    nlist: int
    k: int
    nprobe: int
    delta_d: int
    alpha: float = 0.1
    store: str = "f32"          # stored coordinate type of the index
    seed: int = 0


# The five workloads: plain small / plain at scale / precision / uneven batch / serving.
WORKLOADS = {
    "small-20k-d128": Workload("small-20k-d128", 20_000, 128, 64, 1.2, 100, 64, 10, 8, 32),
    "scale-1m-d128": Workload("scale-1m-d128", 1_000_000, 128, 1024, 1.0, 10_000, 1024, 10, 16, 16),
    "highd-1m-d960": Workload("highd-1m-d960", 1_000_000, 960, 2048, 1.5, 1_000, 4096, 10, 64, 32,
                              store="bf16"),
    "uneven-2m-d256": Workload("uneven-2m-d256", 2_000_000, 256, 4096, 1.2, 4_096, 4096, 100, 128, 32,
                               store="bf16"),
    "serve-5m-d768": Workload("serve-5m-d768", 5_000_000, 768, 8192, 1.3, 1_000, 8192, 10, 32, 32,
                              store="bf16"),
}


def _streams(seed: int) -> dict:
    ss = np.random.SeedSequence(seed)
    return {name: np.random.default_rng(child) for name, child in zip(STREAMS, ss.spawn(len(STREAMS)))}


def spectrum(dim: int, beta: float) -> np.ndarray:
    """Per-component variances lam_i proportional to i**-beta, normalised to mean 1."""
    lam = np.arange(1, dim + 1, dtype=np.float64) ** (-beta)
    return lam * (dim / lam.sum())


def haar_rotation(rng: np.random.Generator, dim: int) -> np.ndarray:
    g = rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def oblivious_rotation(dim: int, seed: int = 0) -> np.ndarray:
    """A seeded Haar-random orthogonal matrix (columns are the axes), drawn from its own stream:
    the data-oblivious transform that the data-aware one is compared with."""
    return haar_rotation(np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=(7919,))), dim)


def _mixture(rng_lab, rng_noise, centres, rot, sqrt_lam, count, chunk=1 << 16):
    """Rows drawn in float32 (noise, scaling and rotation), chunk by chunk."""
    dim = centres.shape[1]
    out = np.empty((count, dim), dtype=np.float32)
    labels = rng_lab.integers(0, centres.shape[0], count)
    rot_t = np.ascontiguousarray(rot.T, dtype=np.float32)
    sl = sqrt_lam.astype(np.float32)
    cen = centres.astype(np.float32)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        z = rng_noise.standard_normal((e - s, dim), dtype=np.float32)
        out[s:e] = cen[labels[s:e]] + (z * sl) @ rot_t
    return out, labels


def make_mixture(n, dim, components, beta, n_queries, seed=0):
    """Return (X [n, dim] float32, Q [n_queries, dim] float32)."""
    st = _streams(seed)
    centres = st["centres"].normal(0.0, 2.0, (components, dim))
    rot = haar_rotation(st["rotation"], dim)
    sqrt_lam = np.sqrt(spectrum(dim, beta))
    X, _ = _mixture(st["labels"], st["noise"], centres, rot, sqrt_lam, n)
    Q, _ = _mixture(st["q_labels"], st["q_noise"], centres, rot, sqrt_lam, n_queries)
    return X, Q


def make(w: Workload, n: int | None = None, n_queries: int | None = None):
    """Base and query sets of a named workload (optionally with fewer rows / queries)."""
    return make_mixture(n or w.n, w.dim, w.components, w.beta, n_queries or w.n_queries, w.seed)


def kmeans_init_rows(n: int, nlist: int, seed: int = 0) -> np.ndarray:
    """nlist distinct row ids, drawn uniformly, used to seed k-means on both sides."""
    rng = _streams(seed)["kmeans_init"]
    return np.sort(rng.choice(n, size=nlist, replace=False)).astype(np.int64)


def calibration_pairs(n: int, n_pairs: int = 100_000, seed: int = 0) -> np.ndarray:
    """[m, 2] int64 ordered pairs (a, b), a != b, uniform over ordered pairs.

    When n*(n-1)/2 <= n_pairs every unordered pair is returned once instead.
    """
    if n < 2:
        return np.zeros((0, 2), dtype=np.int64)
    if n * (n - 1) // 2 <= n_pairs:
        a, b = np.triu_indices(n, 1)
        return np.stack([a, b], 1).astype(np.int64)
    rng = _streams(seed)["calib_pairs"]
    a = rng.integers(0, n, n_pairs)
    b = (a + 1 + rng.integers(0, n - 1, n_pairs)) % n
    return np.stack([a, b], 1).astype(np.int64)


def uneven_batch(n_queries: int, nprobe_lo=8, nprobe_hi=128, ks=(1, 10, 50, 100), seed: int = 0):
    """Per-query (K, nprobe) for the uneven batch: nprobe ~ U{lo..hi}, K ~ U(ks)."""
    rng = _streams(seed)["batch_params"]
    nprobe = rng.integers(nprobe_lo, nprobe_hi + 1, n_queries).astype(np.int32)
    k = np.asarray(ks, dtype=np.int32)[rng.integers(0, len(ks), n_queries)]
    return k, nprobe


def requests(n_requests: int, rate_rps: float, ks=(10, 100), nprobes=(32, 96), seed: int = 0):
    """Poisson arrivals at `rate_rps` requests per second (arrival times in seconds); each request
    holds floor(exp(U[0, ln 257))) clipped to [1, 256] queries and draws its K and nprobe."""
    rng = _streams(seed)["arrivals"]
    gaps = rng.exponential(1.0 / rate_rps, n_requests)
    sizes = np.clip(np.floor(np.exp(rng.uniform(0.0, math.log(257.0), n_requests))), 1, 256).astype(np.int64)
    k = np.asarray(ks)[rng.integers(0, len(ks), n_requests)]
    nprobe = np.asarray(nprobes)[rng.integers(0, len(nprobes), n_requests)]
    return np.cumsum(gaps), sizes, k.astype(np.int32), nprobe.astype(np.int32)
