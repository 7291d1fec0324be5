"""Helpers for the GPU parity tests: compare a device CSC with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle

# float64 runs: 1e-12 relative to sum |a*b| per entry; float32 runs: 1e-5.
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def host_sorted(C):
    """(colptr, rowidx sorted per column, values) of a device CSC, on the host."""
    cp = C.colptr.cpu().numpy().astype(np.int64)
    cp = cp - cp[0]
    ri = C.rowidx.cpu().numpy()
    v = C.values.cpu().numpy().astype(np.float64)
    col = np.repeat(np.arange(cp.size - 1), np.diff(cp))
    order = np.lexsort((ri, col))
    return cp, ri[order], v[order]


def assert_matches(C, P, dtype, what=""):
    """Structure bit-exact (column pointers and per-column sorted rows) and
    values within TOL[dtype] * sum |a*b| (the oracle's absum)."""
    cp, ri, v = host_sorted(C)
    assert cp.size == P.colptr.size, f"{what}: column count"
    assert np.array_equal(cp, P.colptr), f"{what}: column pointers differ"
    assert np.array_equal(ri, P.rowidx), f"{what}: row sets differ"
    tol = TOL[dtype] * P.absum
    err = np.abs(v - P.values)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{what}: {bad.size} values off, worst {float((err / np.maximum(P.absum, 1e-300)).max()):.3e}"
    # every column's rows unique (a lost or duplicated hash insert shows here)
    assert np.all((np.diff(ri) > 0) | (np.diff(np.repeat(np.arange(cp.size - 1), np.diff(cp))) != 0))


def sorted_values(C, values):
    """Values aligned with C's stored entries (device or host), put in the
    per-column row order of host_sorted(C)."""
    cp = C.colptr.cpu().numpy().astype(np.int64)
    cp = cp - cp[0]
    ri = C.rowidx.cpu().numpy()
    col = np.repeat(np.arange(cp.size - 1), np.diff(cp))
    order = np.lexsort((ri, col))
    v = values.cpu().numpy() if isinstance(values, torch.Tensor) else np.asarray(values)
    return v.astype(np.float64)[order]


def grads_and_bounds(A, B, P, dc):
    """Oracle gradients for dC = dc on P(C) (values in the oracle's row
    order), and per gradient entry the sum of |terms| (the scale of the
    float64 and float32 bounds)."""
    dCh = oracle.Mat(P.nrows, P.ncols, P.colptr, P.rowidx, dc)
    gA, gB = oracle.grad_a(A, B, dCh), oracle.grad_b(A, B, dCh)
    adC = oracle.Mat(P.nrows, P.ncols, P.colptr, P.rowidx, np.abs(dc))
    Aa, Ba = oracle.as_mat(A), oracle.as_mat(B)
    sA = oracle.grad_a(Aa, oracle.Mat(Ba.nrows, Ba.ncols, Ba.colptr, Ba.rowidx, np.abs(Ba.values)), adC)
    sB = oracle.grad_b(oracle.Mat(Aa.nrows, Aa.ncols, Aa.colptr, Aa.rowidx, np.abs(Aa.values)), Ba, adC)
    return gA, gB, sA, sB


def assert_grads(A, B, C, dC, dA, dB, dtype, what=""):
    """Device gradients dA, dB of the loss whose dC (device values aligned
    with C's entries) the device used, against the oracle's direct formulas
    on the same dC: every entry within TOL[dtype] * sum |terms|.  C's
    structure must already match the oracle's product."""
    P = oracle.spgemm(A, B)
    gA, gB, sA, sB = grads_and_bounds(A, B, P, sorted_values(C, dC))
    tol = TOL[dtype]
    dA = dA.double().cpu().numpy()
    dB = dB.double().cpu().numpy()
    ea, eb = np.abs(dA - gA), np.abs(dB - gB)
    assert np.all(ea <= tol * sA + 1e-300), f"{what} dA: worst {float((ea / np.maximum(sA, 1e-300)).max()):.3e}"
    assert np.all(eb <= tol * sB + 1e-300), f"{what} dB: worst {float((eb / np.maximum(sB, 1e-300)).max()):.3e}"


def to_dev(M, device="cuda"):
    return M.to(device)


def budget_for_batches(S, eng, plan, nb: int) -> int:
    """Smallest HBM budget for which the planner picks at most nb batches
    (bisection over the memory left to outputs)."""
    total = int((8 * plan.nnz_host[-1] + 8).sum()) * max(1, plan.nnz_host.shape[0] - 1)
    lo, hi, best = total // (nb + 1) + 1, total, None
    while lo <= hi:
        mid = (lo + hi) // 2
        try:
            b, _ = S.plan_batches(plan.nnz_host.reshape(-1), eng.B.ncols, eng.L, eng.vbytes, 0, mid, 0)
        except S.SpgemmError:
            lo = mid + 1
            continue
        if len(b) - 1 > nb:
            lo = mid + 1
        else:
            best, hi = mid, mid - 1
    assert best is not None
    return eng.input_bytes + eng.reserve_bytes + best


def weighted_column_sums_expected(A, B, w):
    """For every column j of C = A B: e_j = sum_i w_i C(i,j), formed as
    (w^T A) B(:,j), and b_j = sum over product terms of |w_i A(i,k) B(k,j)|,
    in float64 on the host.  A property of the product that holds at any
    size: a wrong, missing or repeated row, or a wrong value, in column j
    moves sum_i w_i C(i,j) away from e_j (weights are distinct per row)."""
    A, B = oracle.as_mat(A), oracle.as_mat(B)
    acol = np.repeat(np.arange(A.ncols, dtype=np.int32), np.diff(A.colptr))
    bcol = np.repeat(np.arange(B.ncols, dtype=np.int32), np.diff(B.colptr))
    t = w[A.rowidx] * A.values.astype(np.float64)
    wa = np.bincount(acol, weights=t, minlength=A.ncols)
    wabs = np.bincount(acol, weights=np.abs(t), minlength=A.ncols)
    bv = B.values.astype(np.float64)
    e = np.bincount(bcol, weights=wa[B.rowidx] * bv, minlength=B.ncols)
    b = np.bincount(bcol, weights=wabs[B.rowidx] * np.abs(bv), minlength=B.ncols)
    return e, b


def weighted_column_sums(C, values, w_dev, chunk=1 << 27):
    """sum_i w_i C(i,j) for every column of a device CSC (float64, device
    segment sums over column chunks of at most `chunk` entries)."""
    cp_h = C.colptr.cpu().numpy().astype(np.int64)
    cp_h = cp_h - cp_h[0]
    base = int(C.colptr[0])
    out = torch.zeros(C.ncols, dtype=torch.float64, device=C.rowidx.device)
    lens = (C.colptr[1:] - C.colptr[:-1])
    a = 0
    while a < C.ncols:
        b = a + 1
        hi = np.searchsorted(cp_h, cp_h[a] + chunk, side="right") - 1
        b = max(b, min(C.ncols, int(hi)))
        s, e = base + int(cp_h[a]), base + int(cp_h[b])
        if e > s:
            x = w_dev[C.rowidx[s:e].long()] * values[s:e].double()
            out[a:b] = torch.segment_reduce(x, "sum", lengths=lens[a:b])
        a = b
    return out.cpu().numpy()
