"""Test-side helpers: dense <-> CSC conversion and canonical comparison.

Nothing here computes a product; the tests use these only to build inputs
and to put outputs in a canonical (per-column sorted) order.
"""
from __future__ import annotations

import numpy as np

from oracle import Mat


def dense_to_csc(D, dtype=np.float64, shuffle_seed=None) -> Mat:
    D = np.asarray(D, dtype=np.float64)
    m, n = D.shape
    cp = [0]
    ri, vals = [], []
    rng = np.random.default_rng(shuffle_seed) if shuffle_seed is not None else None
    for j in range(n):
        rows = np.nonzero(D[:, j])[0]
        if rng is not None:
            rows = rng.permutation(rows)
        ri.extend(rows.tolist())
        vals.extend(D[rows, j].tolist())
        cp.append(len(ri))
    return Mat(m, n, np.array(cp, np.int64), np.array(ri, np.int32), np.array(vals, dtype))


def pattern_dense(M) -> np.ndarray:
    P = np.zeros((M.nrows, M.ncols), np.int64)
    for j in range(M.ncols):
        P[M.rowidx[M.colptr[j]:M.colptr[j + 1]], j] = 1
    return P


def csc_to_dense(M, values=None) -> np.ndarray:
    v = M.values if values is None else values
    D = np.zeros((M.nrows, M.ncols), np.float64)
    for j in range(M.ncols):
        s, e = int(M.colptr[j]), int(M.colptr[j + 1])
        D[M.rowidx[s:e], j] = v[s:e]
    return D


def random_sparse(m, n, density, rng, dtype=np.float64, dist="uniform") -> Mat:
    mask = rng.random((m, n)) < density
    if dist == "uniform":
        vals = 1.0 - rng.random((m, n))
    else:
        vals = rng.standard_normal((m, n))
    D = np.where(mask, vals, 0.0)
    M = dense_to_csc(D, dtype, shuffle_seed=int(rng.integers(1 << 30)))
    # re-read values through the pattern so structural entries equal the mask
    return M


def sort_columns(colptr, rowidx, *vals):
    """Per-column sort by row; returns (rowidx, *vals) permuted."""
    colptr = np.asarray(colptr, np.int64)
    rowidx = np.asarray(rowidx)
    ncols = colptr.size - 1
    col = np.repeat(np.arange(ncols, dtype=np.int64), np.diff(colptr))
    order = np.lexsort((rowidx, col))
    return (rowidx[order],) + tuple(np.asarray(v)[order] for v in vals)
