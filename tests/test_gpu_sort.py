"""GPU parity of the row-sorted output option: the sort pass on ragged
synthetic columns (every length class and its boundaries, row windows of
2^19 rows crossed and skipped) against numpy's sort, and sorted products
(plain, batched, layered, tall) whose columns must equal the oracle's,
which emits rows in ascending order, with no sorting on the host."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL

pytestmark = pytest.mark.gpu

S = None


def setup_module(module):
    global S
    import paper_2010_08526_amd as lib
    S = lib


def _ragged(lengths, m, seed, dtype):
    """Columns of the given lengths, distinct rows in random order; rows of
    the long columns spread over the whole of [0, m)."""
    rng = np.random.default_rng(seed)
    cp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    rows = []
    for n in lengths:
        if n > 0:
            span = m if n > 4096 or rng.random() < 0.5 else min(m, 4 * n + 7)
            lo = 0 if span == m else int(rng.integers(0, m - span + 1))
            rows.append((lo + rng.choice(span, n, replace=False)).astype(np.int32))
    ri = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    v = rng.standard_normal(ri.size)
    return synth.CSC(m, len(lengths), torch.from_numpy(cp), torch.from_numpy(ri), torch.from_numpy(v).to(dtype))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_sort_ragged_columns(dtype):
    print(f"case: sort ragged {dtype}", flush=True)
    lengths = [0, 1, 2, 63, 64, 65, 100, 127, 128, 129, 1000, 4095, 4096, 4097, 9000, 70000, 300000, 0, 5, 2048]
    M = _ragged(lengths, 1_200_000, 7, dtype)
    Md = M.to("cuda")
    Sd = S.sort_columns(Md)
    ws = S.alloc_workspace(S.workspace_size(S.OP_SORT, Md))
    Sd2 = S.sort_columns(Md, ws=ws)
    S.check_ws(ws, "sort")
    cp = M.colptr.numpy()
    col = np.repeat(np.arange(M.ncols), np.diff(cp))
    order = np.lexsort((M.rowidx.numpy(), col))
    want_r = M.rowidx.numpy()[order]
    want_v = M.values.numpy()[order]
    for got in (Sd, Sd2):
        assert torch.equal(got.colptr.cpu(), M.colptr)
        assert np.array_equal(got.rowidx.cpu().numpy(), want_r)
        assert np.array_equal(got.values.cpu().numpy(), want_v)  # moved, not recomputed: bit-exact


def test_sort_tall_rows_and_sparse_windows():
    """Long columns in a 9,000,000-row matrix: 18 windows of 2^19 rows, most
    of them empty for the columns concentrated in a few row ranges."""
    print("case: sort tall", flush=True)
    rng = np.random.default_rng(9)
    m = 9_000_000
    cols = []
    for n, span_lo, span in [(50000, 0, m), (6000, 8_500_000, 400_000), (7000, 100, 60_000), (4200, 0, 4200)]:
        cols.append((span_lo + rng.choice(span, n, replace=False)).astype(np.int32))
    cp = np.concatenate([[0], np.cumsum([c.size for c in cols])]).astype(np.int64)
    ri = np.concatenate(cols)
    v = rng.random(ri.size).astype(np.float32)
    M = synth.CSC(m, len(cols), torch.from_numpy(cp), torch.from_numpy(ri), torch.from_numpy(v))
    got = S.sort_columns(M.to("cuda"))
    for j in range(len(cols)):
        s, e = cp[j], cp[j + 1]
        o = np.argsort(ri[s:e], kind="stable")
        assert np.array_equal(got.rowidx[s:e].cpu().numpy(), ri[s:e][o])
        assert np.array_equal(got.values[s:e].cpu().numpy(), v[s:e][o])


def test_sort_reports_repeated_rows():
    """A column with a repeated row (not an output of this library) is
    reported through the workspace status; every write stays inside the
    column."""
    print("case: sort repeated rows", flush=True)
    rows = np.array([5, 3, 5, 1] + list(range(10, 6010)) + [10], np.int32)  # 4 + 6000 + 1 entries, rows 5 and 10 twice
    cp = np.array([0, 4, rows.size], np.int64)
    M = synth.CSC(20000, 2, torch.from_numpy(cp), torch.from_numpy(rows), torch.ones(rows.size))
    guard = torch.full((rows.size + 64,), -7, dtype=torch.int32, device="cuda")
    vout = torch.zeros(rows.size + 64, dtype=torch.float32, device="cuda")
    ws = S.alloc_workspace(S.workspace_size(S.OP_SORT, M))
    S.sort_columns(M.to("cuda"), guard, vout, ws=ws)
    rc, code = S.ws_status_code(ws)
    assert rc == S.E_DEVICE and code == 11
    assert torch.all(guard[rows.size:] == -7)  # nothing written past the matrix


def _assert_sorted_matches(C, P, dtype, what):
    """Columns already in row order: compared with the oracle as they are."""
    cp = C.colptr.cpu().numpy().astype(np.int64)
    cp = cp - cp[0]
    assert np.array_equal(cp, P.colptr), f"{what}: column pointers"
    assert np.array_equal(C.rowidx.cpu().numpy(), P.rowidx), f"{what}: rows (order included)"
    v = C.values.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(v - P.values) <= TOL[dtype] * P.absum), f"{what}: values"


@pytest.mark.parametrize("case", ["er4096", "rmat14_batches", "protein_layers", "tall"])
def test_sorted_products_match_oracle_order(case):
    print(f"case: sorted product {case}", flush=True)
    if case == "er4096":
        A, B = synth.make_workload("er4096")
        dtype, layers, nb = torch.float64, 1, None
    elif case == "rmat14_batches":
        A = synth.rmat(14, 16, 5, dtype=torch.float32)
        B, dtype, layers, nb = A, torch.float32, 1, 5
    elif case == "protein_layers":
        A = synth.protein_like(20000, 11, dtype=torch.float32)
        B, dtype, layers, nb = A, torch.float32, 4, 3
    else:
        from tests.test_gpu_global_heavy import COUNTS, _right, _tall_left
        A = _tall_left(torch.float32, seed=81)
        B = _right(A.ncols, COUNTS, torch.float32, seed=82)
        dtype, layers, nb = torch.float32, 2, None
    Ad, Bd = A.to("cuda"), B.to("cuda")
    eng = S.Engine(Ad, Bd, layers, sorted_output=True)
    if nb is not None:
        from tests.gpu_util import budget_for_batches
        pl = eng.plan()
        eng.budget_bytes = budget_for_batches(S, eng, pl, nb)
    C, plan = eng.run()
    if nb is not None:
        assert plan.nbatches > 1
    _assert_sorted_matches(C, oracle.spgemm(A, B), dtype, case)
