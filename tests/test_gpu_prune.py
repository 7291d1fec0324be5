"""GPU parity of the per-column pruning of an output batch (threshold, then
top-k per column) against the oracle: column pointers, rows and value bits
identical, entry for entry, since selection does no arithmetic."""
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


def _assert_exact(G, P, what):
    cp = G.colptr.cpu().numpy()
    assert np.array_equal(cp, P.colptr), f"{what}: column pointers differ"
    ri = G.rowidx.cpu().numpy()
    assert np.array_equal(ri, P.rowidx), f"{what}: rows differ"
    v = G.values.cpu().numpy().astype(np.float64)
    assert np.array_equal(v.view(np.uint64), P.values.view(np.uint64)), f"{what}: value bits differ"


CASES = [(-np.inf, 1), (-np.inf, 3), (0.0, 2), (0.25, 0), (-0.75, 17), (-np.inf, -1), (1.0, -1), (-1.0, 64),
         (np.nan, 4)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("threshold,k", CASES)
def test_prune_ragged_ties(dtype, threshold, k):
    """104 columns of 0 ... 2100 entries (empty, shorter than k, one to
    three compaction steps of 1024 and their edges), values from 9 levels
    with signed zeros and NaN."""
    print(f"case: prune ragged {dtype} thr={threshold} k={k}", flush=True)
    counts = torch.tensor([0, 1, 2, 300, 255, 256, 257, 1023, 1024, 1025, 2047, 2048, 2049, 2100] +
                          [(37 * i) % 301 for i in range(90)])
    M = synth.tie_heavy(2100, counts, 7, dtype)
    G = S.prune_topk(M.to("cuda"), threshold, k)
    _assert_exact(G, oracle.prune_topk(M, threshold, k), f"{dtype} {threshold} {k}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [1, 100, 69999, 249999, 250000])
def test_prune_long_columns(dtype, k):
    """Columns of 250,000 and 70,000 entries: the select walks every digit of
    long runs of equal values and the compaction spans about 1000 chunks."""
    print(f"case: prune long {dtype} k={k}", flush=True)
    M = synth.tie_heavy(400_000, [0, 250_000, 3, 70_000, 1], 11, dtype, levels=5, nan_frac=0.001)
    for thr in (-np.inf, 0.0):
        G = S.prune_topk(M.to("cuda"), thr, k)
        _assert_exact(G, oracle.prune_topk(M, thr, k), f"long {thr} {k}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_prune_continuous_values(dtype):
    """Few ties: values spread over many binades (the first, 12-bit digit
    splits them finely and the chosen bucket is resolved in LDS) and values
    packed into one binade (the bucket holds too many candidates for LDS and
    the byte digits decide), in columns of 10 ... 120,000 entries."""
    print(f"case: prune continuous {dtype}", flush=True)
    rng = np.random.default_rng(23)
    lens = [10, 150, 2047, 2049, 5000, 40000, 120000, 70000, 3000]
    m = 200_000
    cp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ri = np.concatenate([rng.choice(m, n, replace=False) for n in lens]).astype(np.int32)
    wide = np.exp(rng.uniform(-30, 5, ri.size)) * rng.choice([-1.0, 1.0], ri.size, p=[0.1, 0.9])
    narrow = 1.0 + rng.random(ri.size)  # one binade: [1, 2)
    for name, v in (("wide", wide), ("narrow", narrow)):
        M = synth.CSC(m, len(lens), torch.from_numpy(cp), torch.from_numpy(ri), torch.from_numpy(v).to(dtype))
        for thr, k in ((-np.inf, 1), (0.0, 100), (-np.inf, 1000), (1e-6, 3000)):
            G = S.prune_topk(M.to("cuda"), thr, k)
            _assert_exact(G, oracle.prune_topk(M, thr, k), f"continuous {name} {thr} {k}")


def test_prune_more_columns_than_workgroups():
    """70,000 columns: more than the grid, so workgroups take several columns."""
    print("case: prune 70000 columns", flush=True)
    M = synth.tie_heavy(64, torch.arange(70_000) % 65, 13, torch.float32)
    for thr, k in ((-np.inf, 5), (0.5, 1), (-np.inf, -1)):
        G = S.prune_topk(M.to("cuda"), thr, k)
        _assert_exact(G, oracle.prune_topk(M, thr, k), f"wide {thr} {k}")


def test_prune_empty_matrices():
    print("case: prune empty", flush=True)
    for counts in ([], [0, 0, 0]):
        M = synth.tie_heavy(10, counts, 1, torch.float32)
        G = S.prune_topk(M.to("cuda"), 0.0, 3)
        assert G.colptr.cpu().tolist() == [0] * (len(counts) + 1) and G.nnz == 0


def test_prune_workspace_reuse_across_shapes():
    """One workspace, a large call then a smaller one: per-column state is
    rewritten by each call."""
    print("case: prune workspace reuse", flush=True)
    big = synth.tie_heavy(500, torch.arange(3000) % 501, 17, torch.float64)
    small = synth.tie_heavy(40, torch.arange(50) % 41, 19, torch.float64)
    ws = S.alloc_workspace(S.workspace_size(S.OP_PRUNE, big), "cuda")
    for M, k in ((big, 7), (small, 2), (big, -1)):
        G = S.prune_topk(M.to("cuda"), -1.0, k, ws=ws)
        _assert_exact(G, oracle.prune_topk(M, -1.0, k), f"reuse {M.ncols} {k}")


def test_prune_as_batch_consumer():
    """The consumer of each output batch of C = A*B (integer-valued float64
    inputs, so every product value is exact and ties are common): pruning
    batch by batch gives, column for column, the kept set the oracle finds
    on its own product."""
    print("case: prune consumer", flush=True)
    A = synth.erdos_renyi(3000, 3000, 12, 23, torch.float64)
    A = A.with_values(torch.ceil(A.values * 3))
    Ad = A.to("cuda")
    eng = S.Engine(Ad, Ad, 1, None)
    plan = eng.plan()
    total_out = int((12 * plan.nnz_host[0] + 8).sum())
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + total_out // 4 + int(plan.nnz_host[0].max()) * 12 + 8
    thr, k = 2.0, 6
    kept = []

    def consume(c0, c1, Cb):
        kept.append((c0, c1, S.prune_topk(Cb, thr, k)))

    pl = eng.run(consume=consume)
    assert pl.nbatches >= 3
    P = oracle.prune_topk(oracle.spgemm(A, A), thr, k)
    for c0, c1, G in kept:
        cp, ri, v = host_sorted(G)
        assert np.array_equal(cp, P.colptr[c0:c1 + 1] - P.colptr[c0]), f"batch {c0}:{c1} counts"
        s, e = P.colptr[c0], P.colptr[c1]
        col = np.repeat(np.arange(c1 - c0), np.diff(P.colptr[c0:c1 + 1]))
        order = np.lexsort((P.rowidx[s:e], col))
        assert np.array_equal(ri, P.rowidx[s:e][order]), f"batch {c0}:{c1} rows"
        assert np.array_equal(v, P.values[s:e][order]), f"batch {c0}:{c1} values"


def test_spgemm_topk_keeps_only_pruned_batches():
    """The one-call form: C = A*A formed in at least three batches, each
    pruned as it is formed; the concatenation equals, column for column,
    the oracle's product pruned as a whole (integer-valued float64 inputs,
    so products are exact and ties common)."""
    print("case: spgemm_topk", flush=True)
    A = synth.erdos_renyi(2500, 2500, 10, 29, torch.float64)
    A = A.with_values(torch.ceil(A.values * 3))
    Ad = A.to("cuda")
    eng = S.Engine(Ad, Ad, 1, None)
    plan = eng.plan()
    total_out = int((12 * plan.nnz_host[0] + 8).sum())
    budget = eng.input_bytes + eng.reserve_bytes + total_out // 3 + int(plan.nnz_host[0].max()) * 12 + 8
    del eng
    thr, k = 3.0, 4
    G = S.spgemm_topk(Ad, Ad, thr, k, budget_bytes=budget)
    P = oracle.prune_topk(oracle.spgemm(A, A), thr, k)
    cp, ri, v = host_sorted(G)
    assert np.array_equal(cp, P.colptr)
    col = np.repeat(np.arange(P.ncols), np.diff(P.colptr))
    order = np.lexsort((P.rowidx, col))
    assert np.array_equal(ri, P.rowidx[order]) and np.array_equal(v, P.values[order])
    assert G.nnz <= k * A.ncols


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_prune_first_step_bound(dtype):
    """Columns longer than one select step (2048 entries), built against the
    lower bound the select takes from its first step (the k-th largest of
    the per-thread maxima of entries 0 ... 2047): the largest entries all
    after the first step; the k largest all inside it, with later entries
    tying the k-th at smaller rows; a first step holding fewer than k
    candidates (NaN and values below the threshold); signed zeros and
    negative values in the first step."""
    print(f"case: prune first-step bound {dtype}", flush=True)
    rng = np.random.default_rng(31)
    m = 50_000
    cols = []
    n = 5000
    # largest entries only after the first step
    v = np.concatenate([rng.uniform(0.0, 1.0, 2048), rng.uniform(10.0, 20.0, n - 2048)])
    cols.append(v)
    # the 200 largest inside the first step (5.0, 5.25, ..., 54.75), later
    # entries tying the smallest twelve of them (5.0 ... 7.75)
    v = rng.uniform(0.0, 1.0, n)
    top = rng.choice(2048, 200, replace=False)
    v[top] = 5.0 + 0.25 * np.arange(200)[::-1]
    v[2048 + rng.choice(n - 2048, 40, replace=False)] = 5.0 + (0.25 * np.arange(40)) % 3.0
    cols.append(v)
    # a first step of NaN and small values, candidates later
    v = np.concatenate([np.full(2048, np.nan), rng.uniform(0.0, 1.0, n - 2048)])
    v[rng.choice(2048, 30, replace=False)] = 0.75
    cols.append(v)
    # signed zeros and negatives up front, positives later
    v = np.concatenate([rng.choice([-0.0, 0.0, -1.0, -2.5], 2048), rng.uniform(-1.0, 1.0, n - 2048)])
    cols.append(v)
    # every entry equal
    cols.append(np.full(n, 0.5))
    cp = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int64)
    ri = np.concatenate([rng.permutation(m)[:len(c)] for c in cols]).astype(np.int32)
    vals = torch.from_numpy(np.concatenate(cols)).to(dtype)
    M = synth.CSC(m, len(cols), torch.from_numpy(cp), torch.from_numpy(ri), vals)
    for thr in (-np.inf, 0.5):
        for k in (1, 100, 189, 190, 195, 200, 201, 255, 256, 257, 2047, 2048, 2049):
            G = S.prune_topk(M.to("cuda"), thr, k)
            _assert_exact(G, oracle.prune_topk(M, thr, k), f"first-step bound {thr} {k}")
