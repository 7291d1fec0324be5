"""CPU oracle for the SpGEMM path.  TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package.  It shares no code with the HIP library
and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, float64 dense accumulator,
OpenMP over output columns); this module builds it with gcc and marshals
numpy arrays.  Every function cites the passage it implements:

* ``spgemm``      -- Gustavson's column formula (Sec. II-C); layer ranges of
                     the inner dimension (Sec. III-B, Alg. 2) and output
                     column ranges = batches (Sec. IV-B, Alg. 4).
* ``flops``       -- number of multiplications (Sec. II-A).
* ``masked_xty``  -- (X^T Y) restricted to a pattern; with ``grad_a`` and
                     ``grad_b`` it gives the gradient of a loss on the
                     pattern of C (product rule; not in the paper).
* ``plan_batches``-- the batch-count bound of Eq. (2) and Alg. 3 with one
                     process, written out in Python integers.
* ``prune_topk``  -- the per-column pruning an application applies to each
                     output batch (threshold, then top-k per column; Sec. I,
                     Sec. IV-B, Sec. V-C), in numpy.
* ``spgemm_semiring`` -- the product over another semiring (min-plus,
                     or-and; Sec. II-A), pure Python for small inputs.

Parity status: every function here is pinned by tests in
``tests/test_oracle.py`` against numpy/scipy, closed forms, invariants or
hand-derived fixtures (``prune_topk`` by a hand-worked fixture with ties and
signed zeros and by a sort-free characterisation on tie-heavy inputs). ``plan_batches`` is pinned by a brute-force search over
all contiguous splits (fewest batches, then smallest largest batch); which of
several equally balanced splits it returns is a convention the paper leaves
open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None

i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c into a shared library next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        I64, I32 = ctypes.c_int64, ctypes.c_int
        lib.orc_flops.argtypes = [i64p, i64p, i32p, I64, I64, I64, I64, i64p]
        lib.orc_count.argtypes = [I64, i64p, i32p, i64p, i32p, I64, I64, I64, I64, i64p, I32]
        lib.orc_fill.argtypes = [I64, i64p, i32p, f64p, i64p, i32p, f64p, I64, I64, I64, I64, i64p, i32p, f64p,
                                 ctypes.c_void_p, ctypes.c_void_p, I32]
        lib.orc_masked_xty.argtypes = [I64, i64p, i32p, f64p, i64p, i32p, f64p, I64, i64p, i32p, f64p, I32]
        lib.orc_grad_a.argtypes = [I64, i64p, i32p, I64, i64p, i32p, f64p, I64, i64p, i32p, f64p, f64p]
        lib.orc_grad_b.argtypes = [I64, i64p, i32p, f64p, i64p, i32p, I64, i64p, i32p, f64p, f64p, I32]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().orc_max_threads())


@dataclass
class Mat:
    """numpy CSC: colptr int64[ncols+1], rowidx int32[nnz], values float64[nnz] or None."""

    nrows: int
    ncols: int
    colptr: np.ndarray
    rowidx: np.ndarray
    values: np.ndarray | None

    @property
    def nnz(self) -> int:
        return int(self.rowidx.size)


def _np(x, dtype):
    if x is None:
        return None
    if hasattr(x, "detach"):  # a torch tensor: copy to host memory
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(x), dtype=dtype)


def as_mat(M) -> Mat:
    """Accept any object with nrows/ncols/colptr/rowidx/values (numpy or torch)."""
    if isinstance(M, Mat):
        return M
    return Mat(int(M.nrows), int(M.ncols), _np(M.colptr, np.int64), _np(M.rowidx, np.int32),
               _np(M.values, np.float64))


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")


def flops(A, B, c0: int = 0, c1: int | None = None, klo: int = 0, khi: int | None = None) -> np.ndarray:
    """Per-output-column multiplication count (Sec. II-A), int64[c1-c0]."""
    A, B = as_mat(A), as_mat(B)
    c1 = B.ncols if c1 is None else c1
    khi = A.ncols if khi is None else khi
    out = np.zeros(c1 - c0, np.int64)
    _check(_load().orc_flops(A.colptr, B.colptr, B.rowidx, c0, c1, klo, khi, out))
    return out


@dataclass
class Product:
    """Columns [c0, c1) of A(:,K) B(K,:); rows sorted per column."""

    nrows: int
    ncols: int
    colptr: np.ndarray  # int64 [ncols+1], starts at 0
    rowidx: np.ndarray  # int32
    values: np.ndarray | None  # float64 (exact sum of float64 products, in B order)
    terms: np.ndarray | None  # int32: number of product terms per entry
    absum: np.ndarray | None  # float64: sum of |a*b| per entry

    @property
    def nnz(self) -> int:
        return int(self.rowidx.size)


def count(A, B, c0: int = 0, c1: int | None = None, klo: int = 0, khi: int | None = None,
          nthreads: int = 0) -> np.ndarray:
    """Structural nnz per output column of A(:,K) B(K,:), K = [klo, khi)."""
    A, B = as_mat(A), as_mat(B)
    c1 = B.ncols if c1 is None else c1
    khi = A.ncols if khi is None else khi
    out = np.zeros(c1 - c0, np.int64)
    _check(_load().orc_count(A.nrows, A.colptr, A.rowidx, B.colptr, B.rowidx, c0, c1, klo, khi, out, nthreads))
    return out


def spgemm(A, B, c0: int = 0, c1: int | None = None, klo: int = 0, khi: int | None = None,
           values: bool = True, nthreads: int = 0) -> Product:
    """Columns [c0,c1) of C = A(:,K) B(K,:) with K = [klo,khi) (Sec. II-C
    column formula; the full product when K is everything)."""
    A, B = as_mat(A), as_mat(B)
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    c1 = B.ncols if c1 is None else c1
    khi = A.ncols if khi is None else khi
    cnt = count(A, B, c0, c1, klo, khi, nthreads)
    cp = np.zeros(c1 - c0 + 1, np.int64)
    np.cumsum(cnt, out=cp[1:])
    nnz = int(cp[-1])
    ri = np.zeros(nnz, np.int32)
    if not values:
        # structure only: run the fill with unit values
        Av = np.ones(A.nnz, np.float64)
        Bv = np.ones(B.nnz, np.float64)
    else:
        Av, Bv = A.values, B.values
    v = np.zeros(nnz, np.float64)
    t = np.zeros(nnz, np.int32)
    ab = np.zeros(nnz, np.float64)
    _check(_load().orc_fill(A.nrows, A.colptr, A.rowidx, Av, B.colptr, B.rowidx, Bv, c0, c1, klo, khi, cp, ri, v,
                            t.ctypes.data, ab.ctypes.data, nthreads))
    return Product(A.nrows, c1 - c0, cp, ri, v if values else None, t, ab if values else None)


def masked_xty(X, Y, M, nthreads: int = 0) -> np.ndarray:
    """out(k,j) = sum_i X(i,k) Y(i,j) for each stored (k,j) of M, in M's slot order."""
    X, Y, M = as_mat(X), as_mat(Y), as_mat(M)
    if X.nrows != Y.nrows or M.nrows != X.ncols or M.ncols != Y.ncols:
        raise ValueError("shape mismatch")
    out = np.zeros(M.nnz, np.float64)
    _check(_load().orc_masked_xty(X.nrows, X.colptr, X.rowidx, X.values, Y.colptr, Y.rowidx, Y.values, Y.ncols,
                                  M.colptr, M.rowidx, out, nthreads))
    return out


def grad_a(A, B, dC) -> np.ndarray:
    """dA(i,k) = sum_j dC(i,j) B(k,j) per stored entry of A (dC on P(C))."""
    A, B, dC = as_mat(A), as_mat(B), as_mat(dC)
    out = np.zeros(A.nnz, np.float64)
    _check(_load().orc_grad_a(A.nrows, A.colptr, A.rowidx, A.nnz, B.colptr, B.rowidx, B.values, B.ncols,
                              dC.colptr, dC.rowidx, dC.values, out))
    return out


def grad_b(A, B, dC, nthreads: int = 0) -> np.ndarray:
    """dB(k,j) = sum_i A(i,k) dC(i,j) per stored entry of B."""
    A, B, dC = as_mat(A), as_mat(B), as_mat(dC)
    out = np.zeros(B.nnz, np.float64)
    _check(_load().orc_grad_b(A.nrows, A.colptr, A.rowidx, A.values, B.colptr, B.rowidx, B.ncols, dC.colptr,
                              dC.rowidx, dC.values, out, nthreads))
    return out


def plan_batches(col_bytes, avail_bytes: int) -> list[int]:
    """Column bounds of the batches: the fewest contiguous column ranges
    whose bytes each fit in ``avail_bytes`` (at least the Eq. (2) bound
    ceil(total / avail) with one process), and among those the split whose
    largest batch is smallest; ties broken by packing greedily from the
    left under that smallest cap.  Raises ValueError when ``avail_bytes``
    <= 0 or one column alone exceeds it."""
    col_bytes = [int(x) for x in col_bytes]
    n = len(col_bytes)
    if avail_bytes <= 0:
        raise ValueError("budget does not cover the inputs")
    if any(x > avail_bytes for x in col_bytes):
        raise ValueError("a single column exceeds the budget")

    def greedy(cap):
        bounds, s = [0], 0
        for c, x in enumerate(col_bytes):
            if s + x > cap:
                bounds.append(c)
                s = 0
            s += x
        bounds.append(n)
        return bounds

    b = len(greedy(avail_bytes)) - 1
    total = sum(col_bytes)
    lo = max([0] + col_bytes + [-(-total // b)])
    hi = avail_bytes
    while lo < hi:
        mid = (lo + hi) // 2
        if len(greedy(mid)) - 1 <= b:
            hi = mid
        else:
            lo = mid + 1
    return greedy(lo)


def prune_topk(M, threshold: float, k: int) -> Mat:
    """Column-wise pruning of one output batch, the consumer the paper puts
    right after each batch (Sec. I and Sec. IV-B: the application prunes or
    discards a batch before the next; Markov clustering keeps the top-k
    entries of every column; Sec. V-C: HipMCL prunes column by column).

    Per column: the candidates are the entries whose value is >= threshold
    (compared in float64; NaN is never a candidate).  With k < 0 every
    candidate is kept; otherwise the k largest candidates by value, ties
    between equal values going to the smaller row index (-0.0 equals 0.0).
    Kept entries stay in their input order.  Values come back as float64
    (exact copies of the inputs)."""
    M = as_mat(M)
    colptr = np.zeros(M.ncols + 1, np.int64)
    rows, vals = [], []
    for j in range(M.ncols):
        b, e = int(M.colptr[j]), int(M.colptr[j + 1])
        r, v = M.rowidx[b:e], M.values[b:e]
        cand = np.nonzero(v >= threshold)[0]
        if k >= 0 and cand.size > k:
            vc = np.where(v[cand] == 0.0, 0.0, v[cand])  # one zero
            order = np.lexsort((r[cand], -vc))  # value descending, then row ascending
            cand = np.sort(cand[order[:k]])
        rows.append(r[cand])
        vals.append(v[cand])
        colptr[j + 1] = colptr[j] + cand.size
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return Mat(M.nrows, M.ncols, colptr, cat(rows, np.int32), cat(vals, np.float64))


_SEMIRINGS = {
    # name: (add, multiply)
    "plus_times": (lambda x, y: x + y, lambda a, b: a * b),
    "min_plus": (min, lambda a, b: a + b),
    "or_and": (lambda x, y: 1.0, lambda a, b: 1.0),
}


def spgemm_semiring(A, B, semiring: str) -> Mat:
    """C = A B over a semiring (Sec. II-A: the algorithms apply to any
    semiring since nothing Strassen-like is used): for every (i, j) with at
    least one product term, C(i, j) is the semiring sum over k of
    A(i, k) (x) B(k, j), terms taken in B's order, then A's.  plus_times is
    the ordinary product; min_plus the tropical one (shortest paths);
    or_and the boolean one (every structural entry is 1).  Pure Python,
    for small inputs.  Rows come out sorted per column."""
    add, mul = _SEMIRINGS[semiring]
    A, B = as_mat(A), as_mat(B)
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    colptr = np.zeros(B.ncols + 1, np.int64)
    rows, vals = [], []
    for j in range(B.ncols):
        acc = {}
        for q in range(B.colptr[j], B.colptr[j + 1]):
            kk, bv = int(B.rowidx[q]), float(B.values[q])
            for p in range(A.colptr[kk], A.colptr[kk + 1]):
                i, t = int(A.rowidx[p]), mul(float(A.values[p]), bv)
                acc[i] = add(acc[i], t) if i in acc else t
        for i in sorted(acc):
            rows.append(i)
            vals.append(acc[i])
        colptr[j + 1] = colptr[j] + len(acc)
    return Mat(A.nrows, B.ncols, colptr, np.array(rows, np.int32), np.array(vals, np.float64))
