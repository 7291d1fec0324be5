"""GPU parity of the heavy-column path that uses dense float64 accumulators
in the workspace (output matrices taller than the row-slab path allows,
more than 8,388,608 rows), for the product and for the merge of layer
partials, and reuse of one workspace across calls whose layouts place
different data where those accumulators live."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import assert_matches

pytestmark = pytest.mark.gpu

S = None
TALL = 9_000_000  # above 2048 slabs of 4096 rows


def setup_module(module):
    global S
    import paper_2010_08526_amd as lib
    S = lib


def _hstack(mats, nrows):
    cps, ris, vs, off = [], [], [], 0
    for M in mats:
        cps.append(M.colptr[:-1] + off)
        ris.append(M.rowidx)
        vs.append(M.values)
        off += M.nnz
    cps.append(torch.tensor([off], dtype=torch.int64))
    return synth.CSC(nrows, sum(M.ncols for M in mats), torch.cat(cps), torch.cat(ris), torch.cat(vs))


def _tall_left(dtype, seed=3):
    """9,000,000 x 3000: 2000 columns of 8 rows spread over all rows, 1000
    columns of 8 rows among the first 20,000 (so that products collide)."""
    spread = synth.erdos_renyi(TALL, 2000, 8, seed, dtype)
    dense = synth.erdos_renyi(20_000, 1000, 8, seed + 1, dtype)
    return _hstack([spread, dense], TALL)


def _right(k, counts, dtype, seed=5):
    """k x len(counts): column j holds counts[j] distinct uniform rows."""
    rng = np.random.default_rng(seed)
    cp = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ri = np.concatenate([rng.choice(k, c, replace=False) for c in counts]).astype(np.int32)
    v = (1.0 - rng.random(ri.size)).astype(np.float64)
    return synth.CSC(k, len(counts), torch.from_numpy(cp), torch.from_numpy(ri),
                     torch.from_numpy(v).to(dtype))


COUNTS = [1500, 3, 900, 2000, 40, 1200, 0, 700, 1, 2500, 64, 1100, 800, 17, 3000, 950]


def _product(ws_num, A, B):
    """Symbolic pass, column pointers and one numeric call on ws_num."""
    n = B.ncols
    ws_sym = S.alloc_workspace(S.workspace_size(S.OP_SYMBOLIC, A, B, 0, n, 1))
    ws_scan = S.alloc_workspace(S.workspace_size(S.OP_COLPTR, None, None, 0, n + 1))
    flops = torch.empty(n, dtype=torch.int64, device="cuda")
    nnz = torch.empty((1, n), dtype=torch.int64, device="cuda")
    S.symbolic(A, B, 0, n, 1, flops, nnz, ws_sym)
    cp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    S.colptr(nnz[0], cp, ws_scan)
    total = int(cp[-1])
    ri = torch.empty(max(1, total), dtype=torch.int32, device="cuda")
    v = torch.empty(max(1, total), dtype=A.values.dtype, device="cuda")
    S.numeric(A, B, 0, n, 0, 1, flops, cp, ri, v, ws_num)
    S.check_ws(ws_num, "numeric")
    S.check_ws(ws_sym, "symbolic")
    return S.CSC(A.nrows, n, cp, ri[:total], v[:total])


def _garbage_ws(nbytes):
    ws = S.alloc_workspace(nbytes)
    ws.fill_(0x5A)
    ws[:4096].zero_()
    return ws


@pytest.mark.parametrize("layers,dtype", [(1, torch.float32), (2, torch.float64), (3, torch.float32)])
def test_tall_heavy_columns_global_accumulators(layers, dtype):
    """Heavy columns of a 9,000,000-row product through the global float64
    accumulators: the numeric pass (layers = 1) and the numeric passes of
    each layer followed by the merge (layers > 1), against the oracle."""
    print(f"case: tall heavy layers={layers} {dtype}", flush=True)
    A = _tall_left(dtype)
    B = _right(A.ncols, COUNTS, dtype)
    P = oracle.spgemm(A, B)
    u = np.diff(P.colptr)
    assert int((u > 5120).sum()) >= 4, "the case must hold columns above the LDS bins"
    S.profile_enable(True)
    try:
        C, plan = S.Engine(A.to("cuda"), B.to("cuda"), layers).run()
        rep = S.profile_report()
    finally:
        S.profile_enable(False)
    assert "heavy_global" in rep, sorted(rep)
    assert not any(k.startswith("heavy_items") or k.startswith("merge_items") for k in rep), sorted(rep)
    assert_matches(C, P, dtype, f"tall layers={layers}")


def test_numeric_workspace_reused_across_layouts():
    """One workspace, three numeric calls: a 9,000,000-row product (global
    accumulators), a 100,000-row product (row slabs written where the
    accumulators were), then the tall product again, each against the
    oracle.  The third call must not take the slab data for zeros."""
    print("case: numeric workspace reuse", flush=True)
    At = _tall_left(torch.float32, seed=11)
    Bt = _right(At.ncols, COUNTS, torch.float32, seed=12)
    Bs = synth.rmat(14, 8, 13, dtype=torch.float32)
    As = synth.CSC(100_000, Bs.ncols, Bs.colptr, Bs.rowidx, Bs.values)  # rows below 16384 of 100,000
    n_t, n_s = Bt.ncols, Bs.ncols
    need = max(S.workspace_size(S.OP_NUMERIC, At, Bt, 0, n_t, 1), S.workspace_size(S.OP_NUMERIC, As, Bs, 0, n_s, 1))
    ws = _garbage_ws(need)
    Pt, Ps = oracle.spgemm(At, Bt), oracle.spgemm(As, Bs)
    assert int((np.diff(Ps.colptr) > 5120).sum()) > 0, "the slabbed product must hold heavy columns"
    Atd, Btd, Asd, Bsd = At.to("cuda"), Bt.to("cuda"), As.to("cuda"), Bs.to("cuda")
    assert_matches(_product(ws, Atd, Btd), Pt, torch.float32, "tall, first")
    assert_matches(_product(ws, Asd, Bsd), Ps, torch.float32, "slabbed")
    assert_matches(_product(ws, Atd, Btd), Pt, torch.float32, "tall, after the slabbed call")


def test_masked_product_workspace_reused_across_column_counts():
    """One workspace, masked products out = (X^T Y) o P(M) with heavy columns
    of Y (more than 5120 entries) and different column counts, so the
    dense accumulators sit at different offsets; each against the oracle."""
    print("case: masked product workspace reuse", flush=True)
    m, k = 60_000, 3000
    X = synth.erdos_renyi(m, k, 40, 21, torch.float64)

    def case(counts, seed):
        Y = _right(m, counts, torch.float64, seed)
        M = synth.erdos_renyi(k, len(counts), 50, seed + 1, torch.float64)
        return Y, M

    small = case([6000, 9000, 100, 7000], 31)
    large = case([6000, 20, 8000] + [30] * 3000 + [12000], 41)
    need = max(S.workspace_size(S.OP_MASKED_XTY, X, Y, 0, Y.ncols) for Y, _ in (small, large))
    ws = _garbage_ws(need)
    Xd = X.to("cuda")
    for what, (Y, M) in (("few columns", small), ("many columns", large), ("few columns again", small)):
        got = S.masked_xty(Xd, Y.to("cuda"), M.to("cuda"), ws=ws)
        S.check_ws(ws, what)
        ref = oracle.masked_xty(X, Y, M)
        # scale of each entry: sum over i of |X(i,k) Y(i,j)|
        Xa = synth.CSC(X.nrows, X.ncols, X.colptr, X.rowidx, X.values.abs())
        Ya = synth.CSC(Y.nrows, Y.ncols, Y.colptr, Y.rowidx, Y.values.abs())
        scale = oracle.masked_xty(Xa, Ya, M)
        err = np.abs(got.cpu().numpy() - ref)
        assert np.all(err <= 1e-12 * scale + 1e-300), f"{what}: worst {float((err / np.maximum(scale, 1e-300)).max()):.3e}"
