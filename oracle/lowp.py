"""Stored-coordinate rounding for a low-precision index (not in the paper).

The paper stores the transformed objects once (after Eq. (13)) and states no precision.
The low-precision index stores each rotated coordinate rounded to BF16 or FP16.  The value
that a GPU index holds is the FP32 rotated coordinate rounded to nearest-even in the
narrower format, so the oracle rounds float64 -> float32 -> 16-bit the same way.

The rerank margin delta is a reading: the ceil(0.999 * M)-th smallest relative error
|S_D(stored) - dis^2| / dis^2 over the calibration pairs.
"""
from __future__ import annotations

import numpy as np

from . import estimator


def round_bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via float32; returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def round_f16(x) -> np.ndarray:
    """Round to the nearest IEEE binary16 (ties to even) via float32; returned as float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def store(Y, dtype: str) -> np.ndarray:
    """Coordinates as a ``dtype`` index holds them ("f32", "bf16" or "f16"), as float64."""
    if dtype == "f32":
        return np.asarray(Y, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return round_bf16(Y)
    if dtype == "f16":
        return round_f16(Y)
    raise ValueError(dtype)


def rerank_margin(X, pairs, stored, quantile: float = 0.999) -> float:
    """delta: a high quantile of the relative error of the stored-precision S_D."""
    S, dis2 = estimator.pair_terms(X, None, pairs, stored=stored)
    rel = np.abs(S[:, -1] - dis2) / dis2
    return float(estimator.order_statistic(rel, quantile))
