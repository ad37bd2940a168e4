"""Data-aware orthogonal transform in float64.

Follows the Methodology section:
* Lemma 1: subtracting the mean changes no distance, so the data are centred
  and the zero-mean assumption holds.
* Eq. (10): the optimal W_d maximises tr(W_d^T E[XX^T] W_d) -- PCA, with
  E[XX^T] approximated by all data objects.
* Eq. (11): w_k is the eigenvector of E[XX^T] for the k-th LARGEST eigenvalue.
* Eq. (12): Var(w_k^T X) = lambda_k.
* After Eq. (13): every object is transformed once and stored.

Readings where the paper is silent: E[XX^T] is the 1/N second moment of the
centred data; each eigenvector's sign is fixed so that its entry of largest
magnitude is positive (the first such entry on ties).  Signs do not change any
distance; the rule only makes artifacts comparable.

Data-oblivious comparison (the random orthogonal projection of Figure 1): any orthogonal W
with lambda_k = Var(w_k^T X), the variance along each axis (for the data-aware W these are the
eigenvalues, Eq. (12)).

Pins: orthonormality, distance preservation, trace identity (Lemma 2),
diagonal rotated covariance (Eq. (12)), SVD of the centred data; axis variances equal the
eigenvalues for the data-aware W and sum to the trace for any orthogonal W.
"""
from __future__ import annotations

import numpy as np


def centre(X) -> np.ndarray:
    """E[X] estimated by the mean of all data objects (Lemma 1)."""
    return np.asarray(X, dtype=np.float64).mean(axis=0)


def second_moment(X, mu) -> np.ndarray:
    """E[Y Y^T] for the zero-mean Y = X - E[X], averaged over all N objects (Eq. (10))."""
    Y = np.asarray(X, dtype=np.float64) - mu
    return (Y.T @ Y) / Y.shape[0]


def fix_signs(V) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    lead = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[lead, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return V * sgn


def eig_descending(C):
    """(lambda, W): eigenpairs of the symmetric C, lambda descending (Eq. (11))."""
    lam, V = np.linalg.eigh(np.asarray(C, dtype=np.float64))
    order = np.argsort(-lam, kind="stable")
    return lam[order], fix_signs(V[:, order])


def fit(X):
    """(mu, W, lambda) of the data-aware transform.  Column k of W is w_k."""
    mu = centre(X)
    lam, W = eig_descending(second_moment(X, mu))
    return mu, W, lam


def rotate(X, mu, W) -> np.ndarray:
    """W^T (x - mu) for every row x (stored once; Lemma 1 makes the shift free)."""
    return (np.asarray(X, dtype=np.float64) - mu) @ W


def axis_variances(X, mu, W) -> np.ndarray:
    """Var(w_k^T X) for every column w_k of W: the mean square of the rotated, centred data."""
    Y = rotate(X, mu, W)
    return np.mean(Y * Y, axis=0)
