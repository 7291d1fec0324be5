"""GPU parity of the numeric pass and the merge over the min-plus and or-and
semirings against the oracle's semiring product (pure Python, so the cases
are small): bit-exact structure and values (a min is exact, an or-and entry
is 1, and a min-plus term is one float64 addition on both sides), in every
bin of the numeric pass, through layered merges, and by repeated min-plus
squaring reaching all-pairs shortest paths."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import host_sorted

pytestmark = pytest.mark.gpu

S = None


def setup_module(module):
    global S
    import paper_2010_08526_amd as lib
    S = lib


def teardown_function(fn):
    if S is not None:
        S._lib.spgemm_debug_min_bin(0)


def _int_weights(M, seed, lo=1, hi=9):
    """M with integer values drawn in [lo, hi] (exact in float32 and sums)."""
    rng = np.random.default_rng(seed)
    v = torch.from_numpy(rng.integers(lo, hi + 1, M.nnz).astype(np.float64)).to(M.values.dtype)
    return synth.CSC(M.nrows, M.ncols, M.colptr, M.rowidx, v)


def _assert_exact(C, P, what):
    cp, ri, v = host_sorted(C)
    assert np.array_equal(cp, P.colptr), f"{what}: column pointers"
    assert np.array_equal(ri, P.rowidx), f"{what}: rows"
    want = P.values.astype(np.float32 if C.values.dtype == torch.float32 else np.float64).astype(np.float64)
    bad = np.nonzero(v != want)[0]
    assert bad.size == 0, f"{what}: {bad.size} values differ, first {v[bad[:3]]} vs {want[bad[:3]]}"


def _run(A, B, semiring, layers=1):
    C, _ = S.Engine(A.to("cuda"), B.to("cuda"), layers, semiring=semiring).run()
    return C


@pytest.mark.parametrize("semiring", ["min_plus", "or_and"])
@pytest.mark.parametrize("min_bin", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_bin(semiring, min_bin, dtype):
    """Each bin of the numeric pass forced in turn on an R-MAT product with
    6000 rows (so heavy columns take row slabs: dense and hash items)."""
    print(f"case: semiring {semiring} bin {min_bin} {dtype}", flush=True)
    R = synth.rmat(11, 8, 31, dtype=dtype)
    A = _int_weights(synth.CSC(6000, R.ncols, R.colptr, R.rowidx, R.values), 1)  # rows below 2048 of 6000
    B = _int_weights(synth.erdos_renyi(R.ncols, 300, 40, 32, dtype), 2)
    P = oracle.spgemm_semiring(A, B, semiring)
    S._lib.spgemm_debug_min_bin(min_bin)
    C = _run(A, B, semiring)
    _assert_exact(C, P, f"{semiring} bin {min_bin}")


@pytest.mark.parametrize("semiring", ["min_plus", "or_and", "plus_times"])
def test_heavy_dense_items(semiring):
    """Columns whose terms crowd one row slab (dense slab items), natural bins."""
    print(f"case: semiring {semiring} dense slab items", flush=True)
    Ah = synth.erdos_renyi(8192, 800, 16, 41, torch.float32)
    A = _int_weights(synth.CSC(9000, 800, Ah.colptr, Ah.rowidx, Ah.values), 3)  # rows in slabs 0-1 of 3
    B = _int_weights(synth.erdos_renyi(800, 48, 700, 42, torch.float32), 4)
    P = oracle.spgemm_semiring(A, B, semiring)
    assert int(np.diff(P.colptr).min()) > 5120
    C = _run(A, B, semiring)
    if semiring == "plus_times":
        from tests.gpu_util import assert_matches
        assert_matches(C, oracle.spgemm(A, B), torch.float32, "plus-times dense items")
    else:
        _assert_exact(C, P, f"{semiring} dense items")


@pytest.mark.parametrize("semiring", ["min_plus", "or_and"])
@pytest.mark.parametrize("layers", [2, 3, 7])
def test_layers_merged(semiring, layers):
    """Inner dimension split into layers; the partial products are merged
    with the semiring's addition: light merge columns (an R-MAT product) and
    heavy ones (more than 5120 rows, regrouped by row slab)."""
    print(f"case: semiring {semiring} layers {layers}", flush=True)
    R = synth.rmat(10, 8, 51, dtype=torch.float32)
    A = _int_weights(R, 5)
    P = oracle.spgemm_semiring(A, A, semiring)
    _assert_exact(_run(A, A, semiring, layers), P, f"{semiring} layers {layers} light")
    A = _int_weights(synth.erdos_renyi(20000, 600, 12, 52, torch.float32), 6)
    B = _int_weights(synth.erdos_renyi(600, 40, 600, 53, torch.float32), 7)
    P = oracle.spgemm_semiring(A, B, semiring)
    assert int(np.diff(P.colptr).min()) > 5120
    _assert_exact(_run(A, B, semiring, layers), P, f"{semiring} layers {layers} heavy")


def test_tall_global_accumulators():
    """min-plus and or-and through the global float64 accumulators (more
    than 8,388,608 rows), product and merge."""
    print("case: semiring tall", flush=True)
    from tests.test_gpu_global_heavy import COUNTS, _right, _tall_left
    A = _int_weights(_tall_left(torch.float32, seed=61), 7)
    B = _int_weights(_right(A.ncols, COUNTS, torch.float32, seed=62), 8)
    for semiring in ("min_plus", "or_and"):
        P = oracle.spgemm_semiring(A, B, semiring)
        for layers in (1, 2):
            _assert_exact(_run(A, B, semiring, layers), P, f"tall {semiring} layers {layers}")


def test_min_plus_squaring_reaches_shortest_paths():
    """Repeated min-plus squaring of a weighted digraph with a stored zero
    diagonal: every squaring equals the oracle's, and after ceil(log2 n)
    squarings the result is scipy's all-pairs shortest paths."""
    print("case: min-plus squaring", flush=True)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(71)
    n = 120
    mask = rng.random((n, n)) < 0.03
    np.fill_diagonal(mask, False)
    Wd = np.where(mask, rng.integers(1, 20, (n, n)).astype(np.float64), 0.0)
    pat = mask | np.eye(n, dtype=bool)
    colptr = np.concatenate([[0], np.cumsum(pat.sum(0))]).astype(np.int64)
    rows = np.concatenate([np.nonzero(pat[:, j])[0] for j in range(n)]).astype(np.int32)
    vals = np.concatenate([np.where(np.arange(n)[pat[:, j]] == j, 0.0, Wd[pat[:, j], j]) for j in range(n)])
    M = synth.CSC(n, n, torch.from_numpy(colptr), torch.from_numpy(rows), torch.from_numpy(vals).float())
    steps = int(np.ceil(np.log2(n)))
    for t in range(steps):
        P = oracle.spgemm_semiring(M, M, "min_plus")
        C = _run(M, M, "min_plus")
        _assert_exact(C, P, f"squaring {t}")
        cp, ri, v = host_sorted(C)
        M = synth.CSC(n, n, torch.from_numpy(cp), torch.from_numpy(ri.astype(np.int32)),
                      torch.from_numpy(v).float())
    got = np.full((n, n), np.inf)
    cp = M.colptr.numpy()
    for j in range(n):
        got[M.rowidx.numpy()[cp[j]:cp[j + 1]], j] = M.values.numpy()[cp[j]:cp[j + 1]]
    want = shortest_path(sp.csr_matrix(Wd.T), method="D", directed=True).T
    assert np.array_equal(got, want)
