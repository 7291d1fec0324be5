"""Host-only checks of the C ABI: no GPU needed, no device work launched.

Every call here either runs purely on the host (planner, sizing, status
text) or fails argument validation before anything is enqueued.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch
import pytest

import oracle
import paper_2010_08526_amd as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "spgemm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spgemm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 9
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for code in range(-8, 1):
        assert S.status_string(code) and S.status_string(code) != "unknown status"
    assert S.status_string(-99) == "unknown status"


# ---------------------------------------------------------------- planner
def _mem(nnz_rows, L, vbytes):
    r = 4 + vbytes
    if L == 1:
        return (r * nnz_rows[0] + 8).tolist()
    return (r * nnz_rows[:L].sum(0) + 8 * L + r * nnz_rows[L] + 8).tolist()


@pytest.mark.parametrize("seed", range(40))
def test_planner_matches_oracle_rule(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 300))
    L = int(rng.choice([1, 1, 2, 4, 16]))
    rows = L + 1 if L > 1 else 1
    vb = int(rng.choice([4, 8]))
    nnz = rng.integers(0, 5000, (rows, n)).astype(np.int64)
    if L > 1:  # union count <= sum of layer counts
        nnz[L] = np.minimum(nnz[L], nnz[:L].sum(0))
    mem = _mem(nnz, L, vb)
    inp, res = int(rng.integers(0, 1000)), int(rng.integers(0, 1000))
    lo = max(mem) if mem else 1
    avail = int(rng.integers(lo, lo + sum(mem) + 2))
    bounds, tot = S.plan_batches(nnz.reshape(-1), n, L, vb, inp, inp + res + avail, res, 100000)
    assert bounds == oracle.plan_batches(mem, avail)
    for i in range(len(bounds) - 1):
        assert np.array_equal(tot[i], nnz[:, bounds[i]:bounds[i + 1]].sum(1))


def test_planner_errors():
    nnz = np.array([10, 20, 30], np.int64)
    with pytest.raises(S.SpgemmError) as e:
        S.plan_batches(nnz, 3, 1, 4, 100, 100, 0)  # nothing left for outputs
    assert e.value.status == S.E_BUDGET
    with pytest.raises(S.SpgemmError) as e:
        S.plan_batches(nnz, 3, 1, 4, 0, 200, 0)  # column 2 needs 8*30+8 = 248 > 200
    assert e.value.status == S.E_BUDGET
    with pytest.raises(S.SpgemmError) as e:
        S.plan_batches(nnz, 3, 1, 4, 0, 300, 0, max_batches=1)
    assert e.value.status == S.E_BUDGET
    with pytest.raises(S.SpgemmError) as e:
        S.plan_batches(nnz, 3, 1, 5, 0, 300, 0)
    assert e.value.status == S.E_DTYPE
    b, tot = S.plan_batches(nnz, 3, 1, 4, 0, 10 ** 6, 0)
    assert b == [0, 3] and tot.tolist() == [[60]]
    b, tot = S.plan_batches(np.zeros(0, np.int64), 0, 1, 4, 0, 100, 0)
    assert b == [0, 0]


def test_planner_fits_exactly_at_the_boundary():
    nnz = np.array([1, 1, 1, 1], np.int64)  # 16 bytes per column with float32
    b, _ = S.plan_batches(nnz, 4, 1, 4, 0, 64, 0)
    assert b == [0, 4]
    b, _ = S.plan_batches(nnz, 4, 1, 4, 0, 63, 0)
    assert b == [0, 2, 4]


# ------------------------------------------------------------- validation
class FakeCSC:
    """Descriptor with non-null fake device addresses; validation never reads them."""

    def __init__(self, nrows, ncols, nnz, dtype=S.F32, values=True):
        self.d = S.spgemm_csc(nrows, ncols, nnz, 0x1000, 0x2000, 0x3000 if values else None, dtype)


def _sym(A, B, c0=0, c1=None, L=1, nnz_out=0x5000, ws=None, ws_bytes=1 << 30):
    c1 = B.d.ncols if c1 is None else c1
    return S._lib.spgemm_symbolic(ctypes.byref(A.d) if A else None, ctypes.byref(B.d) if B else None, c0, c1, L,
                                  None, nnz_out, ws, ws_bytes, None)


def test_symbolic_validation_before_launch():
    A, B = FakeCSC(10, 8, 5), FakeCSC(8, 7, 5)
    assert _sym(None, B) == S.E_INVAL
    assert _sym(A, FakeCSC(9, 7, 5)) == S.E_SHAPE
    assert _sym(A, B, c0=3, c1=2) == S.E_INVAL
    assert _sym(A, B, c1=8) == S.E_INVAL
    assert _sym(A, B, L=0) == S.E_INVAL
    assert _sym(A, B, nnz_out=None) == S.E_INVAL
    assert _sym(A, B, ws=None) == S.E_WORKSPACE
    assert _sym(A, B, ws=0x10010) == S.E_WORKSPACE  # not 256-byte aligned
    assert _sym(A, B, ws=0x10000, ws_bytes=16) == S.E_WORKSPACE
    assert _sym(FakeCSC(1 << 31, 8, 5), B) == S.E_OVERFLOW
    bad = FakeCSC(10, 8, -1)
    assert _sym(bad, B) == S.E_INVAL


def test_numeric_and_merge_validation_before_launch():
    A, B = FakeCSC(10, 8, 5), FakeCSC(8, 7, 5, dtype=S.F64)
    lib = S._lib
    r = lib.spgemm_numeric(ctypes.byref(A.d), ctypes.byref(B.d), 0, 7, 0, 1, None, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30,
                           None)
    assert r == S.E_DTYPE  # mixed dtypes
    B2 = FakeCSC(8, 7, 5)
    r = lib.spgemm_numeric(ctypes.byref(A.d), ctypes.byref(B2.d), 0, 7, 2, 2, None, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30,
                           None)
    assert r == S.E_INVAL  # layer >= n_layers
    noval = FakeCSC(10, 8, 5, values=False)
    r = lib.spgemm_numeric(ctypes.byref(noval.d), ctypes.byref(B2.d), 0, 7, 0, 1, None, 0x1, 0x1, 0x1, 0, 0x10000,
                           1 << 30, None)
    assert r == S.E_INVAL  # numeric needs values
    r = lib.spgemm_numeric(ctypes.byref(A.d), ctypes.byref(FakeCSC(8, 7, 5, dtype=7).d), 0, 7, 0, 1, None, 0x1, 0x1,
                           0x1, 0, 0x10000, 1 << 30, None)
    assert r == S.E_DTYPE
    for sr in (-1, 3):  # not a semiring
        assert lib.spgemm_numeric(ctypes.byref(A.d), ctypes.byref(B2.d), 0, 7, 0, 1, None, 0x1, 0x1, 0x1, sr,
                                  0x10000, 1 << 30, None) == S.E_INVAL
        ok = (S.spgemm_csc * 2)(FakeCSC(10, 4, 3).d, FakeCSC(10, 4, 3).d)
        assert lib.spgemm_merge(ok, 2, 0x1, 0x1, 0x1, sr, 0x10000, 1 << 30, None) == S.E_INVAL
    with pytest.raises(ValueError):
        S.semiring_id("max_times")
    assert [S.semiring_id(x) for x in ("plus_times", "min_plus", "or_and", 2)] == [0, 1, 2, 2]
    parts = (S.spgemm_csc * 2)(FakeCSC(10, 4, 3).d, FakeCSC(10, 5, 3).d)
    assert lib.spgemm_merge(parts, 2, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30, None) == S.E_SHAPE
    assert lib.spgemm_merge(parts, 0, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30, None) == S.E_INVAL
    assert lib.spgemm_merge(parts, 4097, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30, None) == S.E_INVAL
    parts = (S.spgemm_csc * 2)(FakeCSC(10, 4, 3).d, FakeCSC(10, 4, 3, dtype=S.F64).d)
    assert lib.spgemm_merge(parts, 2, 0x1, 0x1, 0x1, 0, 0x10000, 1 << 30, None) == S.E_DTYPE
    assert lib.spgemm_colptr(0x1, -1, 0x1, 0x10000, 1 << 20, None) == S.E_INVAL
    assert lib.spgemm_colptr(0x1, 10, None, 0x10000, 1 << 20, None) == S.E_INVAL
    assert lib.spgemm_colptr(0x1, 10, 0x1, 0x10000, 8, None) == S.E_WORKSPACE
    assert lib.spgemm_ws_status(None, None) == S.E_WORKSPACE
    assert lib.spgemm_ws_invalidate(None, None) == S.E_WORKSPACE


def test_workspace_size_depends_on_shapes():
    A, B = FakeCSC(1000, 800, 5), FakeCSC(800, 700, 5)
    out = ctypes.c_size_t()
    for op in (S.OP_SYMBOLIC, S.OP_NUMERIC):
        assert S._lib.spgemm_workspace_size(op, ctypes.byref(A.d), ctypes.byref(B.d), 0, 700, 1, ctypes.byref(out)) == 0
        assert out.value >= 4096 and out.value % 256 == 0
    # heavy accumulators appear only when a column can exceed the LDS bins
    S._lib.spgemm_workspace_size(S.OP_NUMERIC, ctypes.byref(A.d), ctypes.byref(B.d), 0, 700, 1, ctypes.byref(out))
    small = out.value
    Abig = FakeCSC(1 << 20, 800, 5)
    S._lib.spgemm_workspace_size(S.OP_NUMERIC, ctypes.byref(Abig.d), ctypes.byref(B.d), 0, 700, 1, ctypes.byref(out))
    # numeric: int32 slab offsets, (rows / 8192 + 1) per column of A, plus a slabbed copy of A
    assert out.value >= small + 4 * 129 * 800
    # merge keeps dense float64 accumulators for its heavy columns (about 1 GiB)
    S._lib.spgemm_workspace_size(S.OP_MERGE, ctypes.byref(Abig.d), None, 0, 0, 4, ctypes.byref(out))
    assert out.value > (1 << 29)
    assert S._lib.spgemm_workspace_size(99, ctypes.byref(A.d), ctypes.byref(B.d), 0, 700, 1, ctypes.byref(out)) == S.E_INVAL
    assert S._lib.spgemm_workspace_size(S.OP_NUMERIC, ctypes.byref(A.d), ctypes.byref(B.d), 0, 701, 1,
                                        ctypes.byref(out)) == S.E_INVAL
    assert S._lib.spgemm_workspace_size(S.OP_COLPTR, None, None, 0, 1 << 20, 1, ctypes.byref(out)) == 0


def test_backward_validation_before_launch():
    lib = S._lib
    X, Y, M = FakeCSC(10, 8, 5), FakeCSC(10, 7, 5), FakeCSC(8, 7, 5, values=False)
    r = lib.spgemm_masked_xty(ctypes.byref(X.d), ctypes.byref(FakeCSC(11, 7, 5).d), ctypes.byref(M.d), 0x1, 0x10000,
                              1 << 30, None)
    assert r == S.E_SHAPE
    r = lib.spgemm_masked_xty(ctypes.byref(X.d), ctypes.byref(FakeCSC(10, 7, 5, dtype=S.F64).d), ctypes.byref(M.d),
                              0x1, 0x10000, 1 << 30, None)
    assert r == S.E_DTYPE
    r = lib.spgemm_masked_xty(ctypes.byref(X.d), ctypes.byref(Y.d), ctypes.byref(M.d), None, 0x10000, 1 << 30, None)
    assert r == S.E_INVAL
    r = lib.spgemm_masked_xty(ctypes.byref(X.d), ctypes.byref(Y.d), ctypes.byref(M.d), 0x1, None, 1 << 30, None)
    assert r == S.E_WORKSPACE
    assert lib.spgemm_transpose(None, 0x1, 0x1, None, None, 0x10000, 1 << 30, None) == S.E_INVAL
    assert lib.spgemm_transpose(ctypes.byref(X.d), None, 0x1, None, None, 0x10000, 1 << 30, None) == S.E_INVAL
    assert lib.spgemm_transpose(ctypes.byref(X.d), 0x1, 0x1, None, None, 0x10000, 8, None) == S.E_WORKSPACE
    assert lib.spgemm_permute(0x1, 0x1, 10, 9, 0, 0x1, None) == S.E_DTYPE
    assert lib.spgemm_permute(None, 0x1, 10, S.F32, 0, 0x1, None) == S.E_INVAL
    assert lib.spgemm_permute(0x1, 0x1, -1, S.F32, 0, 0x1, None) == S.E_INVAL
    assert lib.spgemm_permute(None, None, 0, S.F32, 0, None, None) == S.OK


def test_bin_caps_validation():
    lib = S._lib
    import numpy as _np
    good = _np.array([16, 64, 256, 1024, 4096], _np.int64)
    assert lib.spgemm_set_bin_caps(1, good.ctypes.data) == S.OK
    assert lib.spgemm_set_bin_caps(1, None) == S.OK
    too_big = _np.array([33, 128, 512, 2048, 5120], _np.int64)
    assert lib.spgemm_set_bin_caps(1, too_big.ctypes.data) == S.E_INVAL
    not_monotone = _np.array([32, 16, 512, 2048, 5120], _np.int64)
    assert lib.spgemm_set_bin_caps(1, not_monotone.ctypes.data) == S.E_INVAL
    assert lib.spgemm_set_bin_caps(2, good.ctypes.data) == S.E_INVAL  # launch shapes: at most 32 per CU
    sym = _np.array([32, 128, 512, 2048, 16384], _np.int64)
    assert lib.spgemm_set_bin_caps(0, sym.ctypes.data) == S.OK
    assert lib.spgemm_set_bin_caps(0, None) == S.OK
    for which in (2, 3):  # workgroups per compute unit of the bin kernels
        ok = _np.array([4, 4, 2, 2, 1], _np.int64)
        assert lib.spgemm_set_bin_caps(which, ok.ctypes.data) == S.OK
        assert lib.spgemm_set_bin_caps(which, _np.array([4, 4, 0, 2, 1], _np.int64).ctypes.data) == S.E_INVAL
        assert lib.spgemm_set_bin_caps(which, _np.array([4, 4, 33, 2, 1], _np.int64).ctypes.data) == S.E_INVAL
        assert lib.spgemm_set_bin_caps(which, None) == S.OK
    assert lib.spgemm_set_bin_caps(4, None) == S.E_INVAL


def _prune(C, k=3, cap=None, thr=0.0, cp=0x5000, ri=0x6000, v=0x7000, ws=None, ws_bytes=1 << 30):
    if cap is None:
        cap = S.prune_bound(C.d.nnz, C.d.ncols, k) if C else 0
    return S._lib.spgemm_prune_topk(ctypes.byref(C.d) if C else None, thr, k, cp, ri, v, cap, ws, ws_bytes, None)


def _prune_ws(C):
    out = ctypes.c_size_t(0)
    assert S._lib.spgemm_workspace_size(S.OP_PRUNE, ctypes.byref(C.d), None, 0, 0, 1, ctypes.byref(out)) == S.OK
    return int(out.value)


def test_prune_validation_before_launch():
    C = FakeCSC(100, 8, 50)
    assert _prune(None) == S.E_INVAL
    assert _prune(C, cp=None) == S.E_INVAL
    assert _prune(C, k=3, cap=23) == S.E_INVAL  # bound min(50, 3 * 8) = 24
    assert _prune(C, k=-1, cap=49) == S.E_INVAL  # no limit: bound nnz
    assert _prune(C, k=100, cap=49) == S.E_INVAL
    assert _prune(C, ri=None) == S.E_INVAL
    assert _prune(C, v=None) == S.E_INVAL
    assert _prune(C, k=0, cap=0, ri=None, v=None) == S.E_WORKSPACE  # nothing to hold: outputs may be NULL
    assert _prune(FakeCSC(100, 8, 50, values=False)) == S.E_INVAL
    assert _prune(FakeCSC(100, 8, 50, dtype=7)) == S.E_DTYPE
    assert _prune(C) == S.E_WORKSPACE
    assert _prune(C, ws=0x10010) == S.E_WORKSPACE
    need = _prune_ws(C)
    assert _prune(C, ws=0x10000, ws_bytes=need - 1) == S.E_WORKSPACE
    # the bound does not overflow for huge k
    assert _prune(C, k=1 << 62, cap=50) == S.E_WORKSPACE
    assert S.prune_bound(50, 8, 1 << 62) == 50 and S.prune_bound(50, 8, 2) == 16 and S.prune_bound(50, 8, -1) == 50


def test_prune_workspace_grows_with_columns():
    a, b = _prune_ws(FakeCSC(10, 1000, 5)), _prune_ws(FakeCSC(10, 2000, 5))
    assert b - a >= 20 * 1000 - 3 * 256  # 8 + 8 + 4 bytes per column, three regions aligned to 256 bytes
    assert _prune_ws(FakeCSC(10, 0, 0)) > 0


# ------------------------------------------------- planner properties (hypothesis)
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402


@settings(max_examples=150, deadline=None)
@given(st.lists(st.integers(0, 400), min_size=1, max_size=60), st.integers(0, 3000), st.integers(0, 3000),
       st.sampled_from([4, 8]))
def test_planner_properties(counts, extra, extra2, vb):
    """Every batch fits, the batches tile the columns in order, a larger
    budget never needs more batches, one batch exactly when everything
    fits, and the count is at least the Eq. (2) bound ceil(total / avail)."""
    nnz = np.array(counts, np.int64)
    n = nnz.size
    mem = (4 + vb) * nnz + 8
    avail = int(mem.max()) + extra
    b, tot = S.plan_batches(nnz, n, 1, vb, 0, avail, 0)
    assert b[0] == 0 and b[-1] == n and all(x < y for x, y in zip(b, b[1:]))
    for i in range(len(b) - 1):
        assert int(mem[b[i]:b[i + 1]].sum()) <= avail
        assert int(tot[i][0]) == int(nnz[b[i]:b[i + 1]].sum())
    nb = len(b) - 1
    assert nb >= -(-int(mem.sum()) // avail)
    assert (nb == 1) == (int(mem.sum()) <= avail)
    b2, _ = S.plan_batches(nnz, n, 1, vb, 0, avail + extra2, 0)
    assert len(b2) - 1 <= nb
    # an input and reserve share moves the budget, not the split
    b3, _ = S.plan_batches(nnz, n, 1, vb, 1000, avail + 1500, 500)
    assert b3 == b


def test_prune_binding_rejects_pattern_only():
    M = S.CSC(4, 2, torch.zeros(3, dtype=torch.int64), torch.zeros(0, dtype=torch.int32), None)
    with pytest.raises(ValueError):
        S.prune_topk(M, 0.0, 1)


def test_noalloc_forward_refuses_inputs_beyond_its_scratch():
    """The allocation-free forward checks its fixed scratch size on the host,
    before any HIP call: a product whose workspace would exceed it is
    refused; shape and dtype errors come first."""
    import paper_2010_08526_amd.batched as Bt
    lib = S._lib
    n = 4_000_000  # 24 bytes of bin lists per column alone exceed the scratch
    A, B = FakeCSC(n, n, 5), FakeCSC(n, n, 5)
    need = ctypes.c_size_t()
    assert lib.spgemm_workspace_size(S.OP_BATCHED_FORWARD, ctypes.byref(A.d), ctypes.byref(B.d), 0, n, 1,
                                     ctypes.byref(need)) == S.OK
    assert need.value > Bt.NOALLOC_SCRATCH_BYTES
    r = lib.spgemm_batched_forward_noalloc(ctypes.byref(A.d), ctypes.byref(B.d), 10, 0x1, 0x1, 0x1, 0x1, 0x1, None)
    assert r == S.E_WORKSPACE
    assert lib.spgemm_batched_forward_noalloc(ctypes.byref(A.d), ctypes.byref(FakeCSC(n + 1, n, 5).d), 10, 0x1, 0x1,
                                              0x1, 0x1, 0x1, None) == S.E_SHAPE
    assert lib.spgemm_batched_forward_noalloc(ctypes.byref(A.d), ctypes.byref(FakeCSC(n, n, 5, dtype=S.F64).d), 10,
                                              0x1, 0x1, 0x1, 0x1, 0x1, None) == S.E_DTYPE


def test_sort_validation_before_launch():
    lib = S._lib
    C = FakeCSC(100, 10, 5)
    need = ctypes.c_size_t()
    assert lib.spgemm_workspace_size(S.OP_SORT, ctypes.byref(C.d), None, 0, 0, 1, ctypes.byref(need)) == S.OK
    assert need.value >= 4096 + 3 * 4 * 10
    assert lib.spgemm_sort_columns(ctypes.byref(C.d), 0x2000, 0x9000, 0x10000, 1 << 20, None) == S.E_INVAL  # in place
    assert lib.spgemm_sort_columns(ctypes.byref(C.d), 0x8000, 0x3000, 0x10000, 1 << 20, None) == S.E_INVAL
    assert lib.spgemm_sort_columns(ctypes.byref(C.d), None, 0x9000, 0x10000, 1 << 20, None) == S.E_INVAL
    assert lib.spgemm_sort_columns(ctypes.byref(C.d), 0x8000, 0x9000, 0x10000, 16, None) == S.E_WORKSPACE
    assert lib.spgemm_sort_columns(ctypes.byref(FakeCSC(100, 10, 5, values=False).d), 0x8000, 0x9000, 0x10000,
                                   1 << 20, None) == S.E_INVAL


def test_numeric_sorted_validation_before_launch():
    lib = S._lib
    A, B = FakeCSC(10, 8, 5), FakeCSC(8, 7, 5)
    a, b = ctypes.byref(A.d), ctypes.byref(B.d)
    big = 1 << 30

    def call(cf=2.0, sr=0, flops=0x100, tri=0x5000, tv=0x6000, ri=0x2000, v=0x3000, c0=0, c1=7, aa=a, bb=b):
        return lib.spgemm_numeric_sorted(aa, bb, c0, c1, flops, 0x1000, ri, v, tri, tv, cf, sr, 0x10000, big, None)

    for sr in (-1, 3):
        assert call(sr=sr) == S.E_INVAL
    for cf in (-1.0, float("nan")):
        assert call(cf=cf) == S.E_INVAL
    assert call(tri=0x2000) == S.E_INVAL  # staging arrays must differ from the outputs
    assert call(tv=0x3000) == S.E_INVAL
    assert call(tri=None) == S.E_INVAL
    assert call(flops=None) == S.E_INVAL  # the choice needs the flops
    assert call(c1=8) == S.E_INVAL
    assert call(bb=ctypes.byref(FakeCSC(8, 7, 5, dtype=S.F64).d)) == S.E_DTYPE
    assert call(bb=ctypes.byref(FakeCSC(9, 7, 5).d)) == S.E_SHAPE
    assert call(aa=ctypes.byref(FakeCSC(10, 8, 5, values=False).d)) == S.E_INVAL
    assert lib.spgemm_numeric_sorted(a, b, 0, 7, 0x100, 0x1000, 0x2000, 0x3000, 0x5000, 0x6000, 2.0, 0, 0x10000, 16,
                                     None) == S.E_WORKSPACE
    # a numeric workspace holds the two extra column lists of the sorted pass
    need = ctypes.c_size_t()
    assert lib.spgemm_workspace_size(S.OP_NUMERIC, a, b, 0, 7, 1, ctypes.byref(need)) == S.OK
    assert need.value >= 4096 + 8 * 4 * 7
