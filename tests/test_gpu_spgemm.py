"""GPU parity of the forward path (symbolic, planner, numeric, merge)
against the CPU oracle, through the C ABI.  Sizes keep the oracle to
seconds while spanning many tiles, every bin and ragged tails."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL, assert_matches, host_sorted

pytestmark = pytest.mark.gpu

S = None


def setup_module(module):
    global S
    import paper_2010_08526_amd as lib
    S = lib
    assert torch.cuda.is_available()


def teardown_function(fn):
    if S is not None:
        S._lib.spgemm_debug_min_bin(0)


def _run(A, B, layers=1, budget=None):
    Ad, Bd = A.to("cuda"), B.to("cuda")
    C, plan = S.Engine(Ad, Bd, layers, budget).run()
    torch.cuda.synchronize()
    return C, plan


def _symbolic(A, B, layers=1):
    Ad, Bd = A.to("cuda"), B.to("cuda")
    n = Bd.ncols
    rows = layers + 1 if layers > 1 else 1
    ws = S.alloc_workspace(S.workspace_size(S.OP_SYMBOLIC, Ad, Bd, 0, n, layers))
    fl = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    nz = torch.full((rows, n), -7, dtype=torch.int64, device="cuda")
    S.symbolic(Ad, Bd, 0, n, layers, fl, nz, ws)
    S.check_ws(ws)
    return fl.cpu().numpy(), nz.cpu().numpy()


# ------------------------------------------------------------- workload 1
def test_er4096_fp64_matches_oracle():
    print("case: er4096 fp64", flush=True)
    A, B = synth.make_workload("er4096")
    fl, nz = _symbolic(A, B)
    assert np.array_equal(fl, oracle.flops(A, B))
    assert int(fl.sum()) == 4096 * 64
    assert np.array_equal(nz[0], oracle.count(A, B))
    C, plan = _run(A, B)
    assert plan.nbatches == 1
    assert_matches(C, oracle.spgemm(A, B), torch.float64, "er4096")


@pytest.mark.parametrize("min_bin", [0, 1, 2, 3, 4, 5])
def test_every_bin_er(min_bin):
    """Each kernel bin forced in turn (columns go to that bin or larger)."""
    print(f"case: forced bin {min_bin} er", flush=True)
    S._lib.spgemm_debug_min_bin(min_bin)
    A = synth.erdos_renyi(6000, 3001, 7, 99, torch.float64)
    B = synth.erdos_renyi(3001, 2999, 5, 98, torch.float64)
    fl, nz = _symbolic(A, B)
    assert np.array_equal(nz[0], oracle.count(A, B))
    C, _ = _run(A, B)
    assert_matches(C, oracle.spgemm(A, B), torch.float64, f"bin{min_bin}")


@pytest.mark.parametrize("min_bin", [0, 3, 4, 5])
def test_every_bin_rmat_fp32(min_bin):
    print(f"case: forced bin {min_bin} rmat13", flush=True)
    S._lib.spgemm_debug_min_bin(min_bin)
    A = synth.rmat(13, 16, 7, dtype=torch.float32)
    fl, nz = _symbolic(A, A)
    assert np.array_equal(fl, oracle.flops(A, A))
    assert np.array_equal(nz[0], oracle.count(A, A))
    C, _ = _run(A, A)
    assert_matches(C, oracle.spgemm(A, A), torch.float32, f"rmat bin{min_bin}")


def test_rmat_scale15_natural_bins_heavy_columns():
    """m = 32768 > the largest LDS bin, so hub columns take the heavy path."""
    print("case: rmat15", flush=True)
    A = synth.rmat(15, 16, 3, dtype=torch.float32)
    fl, nz = _symbolic(A, A)
    assert np.array_equal(nz[0], oracle.count(A, A))
    assert nz[0].max() > 5120  # at least one heavy column
    C, _ = _run(A, A)
    assert_matches(C, oracle.spgemm(A, A), torch.float32, "rmat15")


def test_unsorted_inputs():
    print("case: unsorted", flush=True)
    A = synth.shuffle_within_columns(synth.rmat(12, 16, 5, dtype=torch.float32), 3)
    B = synth.shuffle_within_columns(synth.erdos_renyi(4096, 3000, 11, 4, torch.float32), 4)
    C, _ = _run(A, B)
    assert_matches(C, oracle.spgemm(A, B), torch.float32, "unsorted")


def test_rectangular_and_empty_columns():
    print("case: rectangular", flush=True)
    rng = np.random.default_rng(1)
    m, k, n = 7000, 333, 1500
    from tests.helpers import random_sparse
    A = random_sparse(m, k, 0.01, rng)
    B = random_sparse(k, n, 0.02, rng)  # many empty columns
    A = synth.CSC(m, k, torch.from_numpy(A.colptr), torch.from_numpy(A.rowidx), torch.from_numpy(A.values))
    B = synth.CSC(k, n, torch.from_numpy(B.colptr), torch.from_numpy(B.rowidx), torch.from_numpy(B.values))
    C, _ = _run(A, B)
    assert_matches(C, oracle.spgemm(A, B), torch.float64, "rect")


def test_degenerate_empty():
    print("case: empty", flush=True)
    Z = synth.CSC(50, 40, torch.zeros(41, dtype=torch.int64), torch.zeros(0, dtype=torch.int32),
                  torch.zeros(0, dtype=torch.float32))
    B = synth.erdos_renyi(40, 30, 3, 1, torch.float32)
    C, plan = _run(Z, B)
    assert C.nnz == 0 and C.colptr.cpu().tolist() == [0] * 31
    C, plan = _run(B, synth.CSC(30, 0, torch.zeros(1, dtype=torch.int64), torch.zeros(0, dtype=torch.int32),
                                 torch.zeros(0, dtype=torch.float32)))
    assert C.ncols == 0


def test_single_term_products_bit_exact():
    """A*I = A and A*diag(s): each entry is one product, correctly rounded."""
    print("case: single-term", flush=True)
    A = synth.rmat(12, 8, 2, dtype=torch.float32)
    n = A.ncols
    I = synth.CSC(n, n, torch.arange(n + 1, dtype=torch.int64), torch.arange(n, dtype=torch.int32),
                  torch.ones(n, dtype=torch.float32))
    C, _ = _run(A, I)
    cp, ri, v = host_sorted(C)
    assert np.array_equal(cp, A.colptr.numpy()) and np.array_equal(ri, A.rowidx.numpy())
    assert np.array_equal(v.astype(np.float32), A.values.numpy())
    s = torch.from_numpy(np.random.default_rng(0).standard_normal(n).astype(np.float32))
    D = I.with_values(s)
    C, _ = _run(A, D)
    cp, ri, v = host_sorted(C)
    ref = (A.values * s[A.col_index()]).numpy()  # float32 product, correctly rounded
    assert np.array_equal(v.astype(np.float32), ref)


@pytest.mark.parametrize("nb_target", [2, 4, 7])
def test_batched_equals_unbatched(nb_target):
    """Batches are column ranges of C (Alg. 4); their concatenation is C."""
    print(f"case: batches {nb_target}", flush=True)
    A = synth.rmat(13, 16, 11, dtype=torch.float32)
    Ad = A.to("cuda")
    eng = S.Engine(Ad, Ad, 1, None)
    plan = eng.plan()
    total_out = int((8 * plan.nnz_host[0] + 8).sum())
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + total_out // nb_target + int(plan.nnz_host[0].max()) * 8 + 8
    C, plan = eng.run()
    assert plan.nbatches >= nb_target
    assert_matches(C, oracle.spgemm(A, A), torch.float32, f"b={plan.nbatches}")


@pytest.mark.parametrize("scale,L", [(12, 2), (12, 3), (12, 16), (9, 600)])
def test_layers_counts_and_merge(scale, L):
    """Per-layer symbolic counts equal the oracle's layer products, and the
    merge of the layer partials equals C (Eq. 1; Merge-Fiber).  L = 600 >
    k = 512 leaves empty layers and merges more than 64 parts."""
    print(f"case: layers {L}", flush=True)
    A = synth.rmat(scale, 16, 13, dtype=torch.float32)
    fl, nz = _symbolic(A, A, L)
    for l, (klo, khi) in enumerate(S.layer_bounds(A.ncols, L)):
        assert np.array_equal(nz[l], oracle.count(A, A, klo=klo, khi=khi)), f"layer {l}"
    assert np.array_equal(nz[L], oracle.count(A, A))
    assert int(fl.sum()) >= int(nz[:L].sum()) >= int(nz[L].sum())
    C, _ = _run(A, A, L)
    assert_matches(C, oracle.spgemm(A, A), torch.float32, f"L={L}")


def test_layers_with_batches_protein_like():
    print("case: protein layers+batches", flush=True)
    A = synth.protein_like(30000, 17)
    Ad = A.to("cuda")
    eng = S.Engine(Ad, Ad, 4, None)
    plan = eng.plan()
    L = 4
    mem = int((8 * plan.nnz_host[:L].sum(0) + 32 + 8 * plan.nnz_host[L] + 8).sum())
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + mem // 3
    C, plan = eng.run()
    assert plan.nbatches >= 3
    assert_matches(C, oracle.spgemm(A, A), torch.float32, "protein")


@pytest.mark.parametrize("which", ["protein", "rmat", "rmat_many_parts", "rmat_300_parts"])
def test_merge_heavy_buckets_forced(which):
    """Every merge column through the heavy path (slab buckets, dense and hash
    items); with 70 layers the parts span more than one chunk of 64, with 300
    more than one group of 256 part ranges staged in LDS."""
    print(f"case: merge buckets {which}", flush=True)
    if which == "protein":
        A, L = synth.protein_like(20000, 23), 3
    elif which == "rmat":
        A, L = synth.rmat(13, 16, 29, dtype=torch.float32), 5
    elif which == "rmat_many_parts":
        A, L = synth.rmat(13, 16, 31, dtype=torch.float32), 70
    else:
        A, L = synth.rmat(13, 16, 37, dtype=torch.float32), 300
    Ad = A.to("cuda")
    eng = S.Engine(Ad, Ad, L, None)
    pl = eng.plan()  # symbolic in the natural bins
    S._lib.spgemm_debug_min_bin(5)
    C = []
    for i in range(pl.nbatches):
        Cb = eng.run_batch(pl, i)
        C.append(synth.CSC(Cb.nrows, Cb.ncols, Cb.colptr.clone(), Cb.rowidx.clone(), Cb.values.clone()))
    S._lib.spgemm_debug_min_bin(0)
    eng.check()
    Cc = S._concat(C, A.nrows)
    assert_matches(Cc, oracle.spgemm(A, A), torch.float32, f"merge buckets {which}")


def test_symbolic_column_range():
    print("case: column range", flush=True)
    A = synth.rmat(12, 16, 21, dtype=torch.float32)
    Ad = A.to("cuda")
    ws = S.alloc_workspace(S.workspace_size(S.OP_SYMBOLIC, Ad, Ad, 1000, 3333, 1))
    fl = torch.empty(2333, dtype=torch.int64, device="cuda")
    nz = torch.empty(2333, dtype=torch.int64, device="cuda")
    S.symbolic(Ad, Ad, 1000, 3333, 1, fl, nz, ws)
    assert np.array_equal(fl.cpu().numpy(), oracle.flops(A, A, 1000, 3333))
    assert np.array_equal(nz.cpu().numpy(), oracle.count(A, A, 1000, 3333))


def test_colptr_scan_large():
    print("case: scan", flush=True)
    rng = np.random.default_rng(0)
    for n in (1, 8191, 8192, 8193, 1_000_003):
        x = rng.integers(0, 1 << 33, n).astype(np.int64)
        d = torch.from_numpy(x).cuda()
        out = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        ws = S.alloc_workspace(S.workspace_size(S.OP_COLPTR, None, None, 0, n))
        S.colptr(d, out, ws)
        ref = np.concatenate([[0], np.cumsum(x)])
        assert np.array_equal(out.cpu().numpy(), ref)


def test_heavy_columns_tall_matrix_two_windows():
    """m = 1.5M rows: heavy columns span two counting windows and 184 row
    slabs; u_j ~ 12000 > the largest LDS bin."""
    print("case: tall heavy", flush=True)
    A = synth.erdos_renyi(1_500_000, 2000, 30, 31, torch.float32)
    B = synth.erdos_renyi(2000, 64, 400, 32, torch.float32)
    fl, nz = _symbolic(A, B)
    assert np.array_equal(nz[0], oracle.count(A, B))
    assert nz[0].min() > 5120
    C, _ = _run(A, B)
    assert_matches(C, oracle.spgemm(A, B), torch.float32, "tall")


@pytest.mark.parametrize("layers", [1, 4])
def test_b_rows_outside_inner_dimension_flagged(layers):
    """A row of B at or beyond k = ncols(A) is reported by the device-side
    check (code 1), by the symbolic pass and, with layers, by each layer's
    split of B in the symbolic and numeric passes; A's column pointers are
    never read for it."""
    print(f"case: bad B row, layers {layers}", flush=True)
    A = synth.erdos_renyi(512, 512, 8, 5, torch.float32)
    B = synth.erdos_renyi(512, 300, 6, 6, torch.float32)
    ri = B.rowidx.clone()
    ri[17] = 512 + 40  # rows within the column stay distinct
    Ad, Bd = A.to("cuda"), B.to("cuda")
    Bbad = synth.CSC(B.nrows, B.ncols, Bd.colptr, ri.to("cuda"), Bd.values)
    n = B.ncols
    rows = layers + 1 if layers > 1 else 1
    ws = S.alloc_workspace(S.workspace_size(S.OP_SYMBOLIC, Ad, Bd, 0, n, layers))
    fl = torch.zeros(n, dtype=torch.int64, device="cuda")
    nz = torch.zeros((rows, n), dtype=torch.int64, device="cuda")
    S.symbolic(Ad, Bbad, 0, n, layers, fl, nz, ws)
    assert S.ws_status_code(ws) == (S.E_DEVICE, 1)
    # numeric of layer 0 with the output layout of the valid B
    _, nz_ok = _symbolic(A, B, layers)
    cnt = torch.from_numpy(nz_ok[0]).to("cuda")
    cp = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    cp[1:] = torch.cumsum(cnt, 0)
    total = int(cp[-1])
    c_ri = torch.full((total + 64,), -5, dtype=torch.int32, device="cuda")
    c_v = torch.zeros(total + 64, dtype=torch.float32, device="cuda")
    wsn = S.alloc_workspace(S.workspace_size(S.OP_NUMERIC, Ad, Bd, 0, n, layers))
    S.numeric(Ad, Bbad, 0, n, 0, layers, fl, cp, c_ri, c_v, wsn)
    assert S.ws_status_code(wsn) == (S.E_DEVICE, 1)
    assert torch.all(c_ri[total:] == -5)  # nothing written past the output


def test_one_column_per_batch():
    """b = ncols: A = 2 I and three entries per column of B, so every column
    of C holds exactly three entries and a budget of one column's bytes
    gives one batch per column; the concatenation equals C."""
    print("case: one column per batch", flush=True)
    n = 150
    B = synth.erdos_renyi(n, n, 3, 37, torch.float32)
    A = synth.CSC(n, n, torch.arange(n + 1, dtype=torch.int64), torch.arange(n, dtype=torch.int32),
                  torch.full((n,), 2.0, dtype=torch.float32))
    eng = S.Engine(A.to("cuda"), B.to("cuda"), 1, None)
    eng.plan()
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + 3 * 8 + 8
    C, plan = eng.run()
    assert plan.nbatches == n
    P = oracle.spgemm(A, B)
    assert_matches(C, P, torch.float32, "b = ncols")
    cp, ri, v = host_sorted(C)
    assert np.array_equal(v, P.values)  # single-term products are exact


@pytest.mark.parametrize("layers", [2, 6])
def test_merge_long_columns_in_two_halves(layers):
    """Merge columns of more than 65,536 partial entries are bucketed as two
    tasks, one per half of the row slabs (the upper half placed against the
    end of the column's bucket range): long columns beside short ones, over
    an odd number of slabs, against the oracle."""
    print(f"case: merge long columns, {layers} layers", flush=True)
    from tests.test_gpu_global_heavy import _right
    m = 300_000  # 74 slabs of 4096 rows
    A = synth.erdos_renyi(m, 400, 400, 111, torch.float32)
    B = _right(400, [400, 3, 350, 0, 200, 399, 60, 1, 380], torch.float32, seed=112)
    P = oracle.spgemm(A, B)
    parts = sum(np.diff(oracle.spgemm(A, B, klo=l * (400 // layers), khi=(l + 1) * (400 // layers)).colptr)
                for l in range(layers))
    assert int(parts.max()) >= 65536  # long columns exist
    C, plan = S.Engine(A.to("cuda"), B.to("cuda"), layers, None).run()
    assert_matches(C, P, torch.float32, f"merge long columns L={layers}")
