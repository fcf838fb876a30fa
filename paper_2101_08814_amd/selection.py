"""Feature selection for computing only some invariants (Sec. 4.H).

Host-side, offline: pick columns of a [samples, features] matrix of power
spectra by farthest-point sampling or by iterative CUR, and translate packed feature columns
into the (k1, k2, l) triples that ``Calculator.power_spectrum_selected``
takes.  Packed layout: column l * K(K+1)/2 + kk, with kk running over
k1 <= k2 row by row (k = species * nmax + n).
"""
from __future__ import annotations

import numpy as np


def fps_columns(X: np.ndarray, n_select: int, first: int | None = None) -> np.ndarray:
    """Farthest-point sampling over the columns of X [samples, features]:
    start from ``first`` (default: the column of largest norm), then
    repeatedly take the column farthest, in Euclidean distance over the
    samples, from every column taken so far (ties: lowest index)."""
    X = np.asarray(X, dtype=np.float64)
    n_feat = X.shape[1]
    if not 0 < n_select <= n_feat:
        raise ValueError(f"n_select must be in [1, {n_feat}]")
    cols = X.T
    sq = np.einsum("ij,ij->i", cols, cols)
    start = int(np.argmax(sq)) if first is None else int(first)
    picked = [start]
    d2 = sq + sq[start] - 2.0 * cols @ cols[start]
    d2[start] = -1.0
    for _ in range(n_select - 1):
        nxt = int(np.argmax(d2))
        picked.append(nxt)
        d2 = np.minimum(d2, sq + sq[nxt] - 2.0 * cols @ cols[nxt])
        d2[picked] = -1.0
    return np.asarray(picked, dtype=np.int64)


def packed_to_triples(n_channels: int, lmax: int, columns) -> np.ndarray:
    """(k1, k2, l) int32 [n, 3] of packed feature columns."""
    K = int(n_channels)
    KK = K * (K + 1) // 2
    k1_of, k2_of = np.triu_indices(K)
    cols = np.asarray(columns, dtype=np.int64)
    if cols.size and (cols.min() < 0 or cols.max() >= (lmax + 1) * KK):
        raise ValueError("feature column out of range")
    l, kk = np.divmod(cols, KK)
    return np.stack([k1_of[kk], k2_of[kk], l], axis=1).astype(np.int32)


def cur_columns(X: np.ndarray, n_select: int, k: int = 1) -> np.ndarray:
    """Iterative CUR column selection: take the column with the largest
    leverage score (squared norm of its entries in the top-k right singular
    vectors of the current matrix), project every column onto the
    orthogonal complement of the chosen one, and repeat on the residual
    (ties: lowest index)."""
    R = np.array(X, dtype=np.float64, copy=True)
    n_feat = R.shape[1]
    if not 0 < n_select <= n_feat:
        raise ValueError(f"n_select must be in [1, {n_feat}]")
    picked = []
    for _ in range(n_select):
        _, _, vt = np.linalg.svd(R, full_matrices=False)
        score = (vt[:k] ** 2).sum(axis=0)
        score[picked] = -1.0
        j = int(np.argmax(score))
        picked.append(j)
        v = R[:, j]
        nv = float(v @ v)
        if nv > 0.0:
            R -= np.outer(v, (v @ R) / nv)
    return np.asarray(picked, dtype=np.int64)
