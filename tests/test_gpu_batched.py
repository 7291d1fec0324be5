"""GPU parity of the batched (block-diagonal, graph-capturable) path."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL, assert_grads, assert_matches, host_sorted

pytestmark = pytest.mark.gpu

S = Bt = None


def setup_module(module):
    global S, Bt
    import paper_2010_08526_amd as lib
    import paper_2010_08526_amd.batched as bt
    S, Bt = lib, bt


def teardown_function(fn):
    if S is not None:
        S._lib.spgemm_debug_min_bin(0)
        for which in range(4):
            Bt.set_bin_caps(which, None)


def _instance(M, off, i):
    """Instance i of a packed block-diagonal matrix, rows made local."""
    o0, o1 = int(off[i]), int(off[i + 1])
    cp = M.colptr[o0:o1 + 1]
    s, e = int(cp[0]), int(cp[-1])
    return synth.CSC(o1 - o0, o1 - o0, (cp - s).contiguous(), (M.rowidx[s:e] - o0).contiguous(),
                     None if M.values is None else M.values[s:e].contiguous())


def _batch(count=48, seed=5, dtype=torch.float32):
    spec = synth.batch_spec(count, seed, nmin=64, nmax=4096)
    return synth.batch_packed(spec, seed, dtype, "cuda")


def test_pack_matches_generator():
    print("case: pack", flush=True)
    A, B, off = _batch(20)
    inst = [_instance(A, off, i) for i in range(20)]
    P, offs = Bt.batch_pack(inst)
    assert torch.equal(P.colptr, A.colptr) and torch.equal(P.rowidx, A.rowidx) and torch.equal(P.values, A.values)
    assert offs[:, 0].tolist() == off.cpu().tolist() and offs[:, 1].tolist() == off.cpu().tolist()


def test_batched_forward_per_instance_oracle_and_plain():
    print("case: batched forward", flush=True)
    A, B, off = _batch(48)
    eng = Bt.BatchedEngine(A, B)
    eng.forward()
    eng.check()
    C = eng.C
    for i in range(0, 48, 5):
        Ai, Bi = _instance(A, off, i), _instance(B, off, i)
        Ci = _instance(C, off, i)
        assert_matches(Ci, oracle.spgemm(Ai.to("cpu"), Bi.to("cpu")), torch.float32, f"instance {i}")
        Cp, _ = S.Engine(Ai, Bi, 1).run()  # the plain path on the same instance
        a, b = host_sorted(Ci), host_sorted(Cp)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.allclose(a[2], b[2], rtol=1e-6, atol=0)


def test_graph_replays_idempotent():
    print("case: graph replay", flush=True)
    A, B, off = _batch(32, seed=9)
    eng = Bt.BatchedEngine(A, B)
    eng.forward()
    torch.cuda.synchronize()
    ref = host_sorted(eng.C)
    eng.capture(eng.forward)
    for rep in range(4):
        eng.values.zero_()
        eng.rowidx.fill_(-1)
        torch.cuda.synchronize()
        eng.replay()
        torch.cuda.synchronize()
        x = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays
        got = host_sorted(eng.C)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), f"replay {rep}"
        assert np.allclose(got[2], ref[2], rtol=1e-6, atol=0), f"replay {rep}"
        assert float(x) == 1000.0
    eng.check()


def test_fused_backward_vs_oracle_and_transpose_path():
    print("case: fused backward", flush=True)
    A, B, off = _batch(24, seed=13, dtype=torch.float64)
    eng = Bt.BatchedEngine(A, B, backward=True)
    eng.forward()
    C = eng.C
    col = torch.repeat_interleave(torch.arange(C.ncols, device="cuda"), C.colptr[1:] - C.colptr[:-1])
    T = synth.target_values(C.rowidx, col, C.ncols, 3, torch.float64)
    dC = (C.values - T).contiguous()
    dA, dB = eng.backward(dC)
    eng.check()
    bw = S.Backward(A, B, C)
    tA, tB = bw(dC)
    assert torch.allclose(dA, tA, rtol=1e-11, atol=1e-12) and torch.allclose(dB, tB, rtol=1e-11, atol=1e-12)
    # against the oracle's direct formulas on the same dC, every entry
    # within 1e-12 * sum |terms|
    Ah, Bh = A.to("cpu"), B.to("cpu")
    assert_matches(C, oracle.spgemm(Ah, Bh), torch.float64, "fused forward")
    assert_grads(Ah, Bh, C, dC, dA, dB, torch.float64, "fused backward")
    assert_grads(Ah, Bh, C, dC, tA, tB, torch.float64, "transpose-based backward")


def test_capacity_overflow_is_reported_and_bounded():
    print("case: overflow", flush=True)
    A, B, off = _batch(8, seed=21)
    eng = Bt.BatchedEngine(A, B)
    full = eng.nnz_c
    guard = torch.full((4096,), -7, dtype=torch.int32, device="cuda")
    eng.nnz_c = full // 2  # claim a smaller capacity than needed
    rowbuf = torch.empty(eng.nnz_c + 4096, dtype=torch.int32, device="cuda")
    rowbuf[eng.nnz_c:] = guard
    eng.rowidx = rowbuf
    eng.forward()
    assert S.ws_status(eng.ws) == S.E_DEVICE
    assert torch.equal(rowbuf[eng.nnz_c:], guard)  # nothing written past the capacity


@pytest.mark.parametrize("min_bin", [2, 4, 5])
def test_batched_forced_bins(min_bin):
    """Forced larger bins in the graph-capturable path, heavy (row slabs)
    included."""
    print(f"case: batched bin {min_bin}", flush=True)
    A, B, off = _batch(16, seed=17)
    S._lib.spgemm_debug_min_bin(min_bin)
    eng = Bt.BatchedEngine(A, B)
    eng.forward()
    eng.check()
    C = eng.C
    P = oracle.spgemm(A.to("cpu"), B.to("cpu"))
    assert_matches(C, P, torch.float32, f"forced {min_bin}")


def test_autotune_changes_speed_not_results():
    print("case: autotune", flush=True)
    A, B, off = _batch(32, seed=23)
    eng = Bt.BatchedEngine(A, B)
    eng.forward()
    torch.cuda.synchronize()
    ref = host_sorted(eng.C)
    res = Bt.autotune(eng, reps=1, use_cache=False)
    assert tuple(res["caps"]) in Bt._candidates()
    assert tuple(res["num_bpc"]) in Bt._bpc_candidates(Bt.NUM_BPC)
    assert tuple(res["sym_bpc"]) in Bt._bpc_candidates(Bt.SYM_BPC)
    assert len(res["tried"]) >= 5
    for t in res["tried"]:
        Bt._apply({"caps": t["caps"], "num_bpc": t["num_bpc"], "sym_bpc": t["sym_bpc"]})
        eng.forward()
        got = host_sorted(eng.C)
        assert np.array_equal(got[1], ref[1]) and np.allclose(got[2], ref[2], rtol=1e-6, atol=0)


def test_fused_backward_skewed_rmat():
    """Fused backward on a skewed product: hub columns of A (64 or more
    entries, walked by the whole wave) next to short ones (flattened into
    rounds) in the same chunks of B(:,j)."""
    print("case: fused backward rmat", flush=True)
    Ah = synth.rmat(12, 8, 41, dtype=torch.float64)
    A = Ah.to("cuda")
    assert int(np.diff(Ah.colptr.numpy()).max()) >= 64
    eng = Bt.BatchedEngine(A, A, backward=True)
    eng.forward()
    C = eng.C
    col = torch.repeat_interleave(torch.arange(C.ncols, device="cuda"), C.colptr[1:] - C.colptr[:-1])
    T = synth.target_values(C.rowidx, col, C.ncols, 5, torch.float64)
    dC = (C.values - T).contiguous()
    dA, dB = eng.backward(dC)
    eng.check()
    tA, tB = S.Backward(A, A, C)(dC)
    assert torch.allclose(dA, tA, rtol=1e-11, atol=1e-12) and torch.allclose(dB, tB, rtol=1e-11, atol=1e-12)
    assert_matches(C, oracle.spgemm(Ah, Ah), torch.float64, "fused forward rmat")
    assert_grads(Ah, Ah, C, dC, dA, dB, torch.float64, "fused backward rmat")
    assert_grads(Ah, Ah, C, dC, tA, tB, torch.float64, "transpose-based backward rmat")


def test_spgemm_batched_one_call_rectangular():
    """The one-call form on uneven square instances and on rectangular ones
    (A_i m_i x k_i, B_i k_i x n_i): each C_i, rows local to its instance,
    against the oracle; graph replay and plain forward agree bit for bit."""
    print("case: spgemm_batched one call", flush=True)
    spec = synth.batch_spec(10, 31, nmin=64, nmax=3000)
    pairs = [synth.batch_instance(spec, i, 31) for i in range(10)]
    shapes = [(300, 40, 2, 1), (7, 500, 3, 2), (1000, 1000, 5, 3), (50, 1, 1, 4)]
    for m, k, d, s in shapes:
        n = 2 * k + 3
        pairs.append((synth.erdos_renyi(m, k, min(d, m), 100 + s, torch.float32),
                      synth.erdos_renyi(k, n, min(d, k), 200 + s, torch.float32)))
    dev = [(a.to("cuda"), b.to("cuda")) for a, b in pairs]
    Cs, _ = Bt.spgemm_batched(dev, graph=True)
    Cp, _ = Bt.spgemm_batched(dev, graph=False)
    for i, ((a, b), C, Q) in enumerate(zip(pairs, Cs, Cp)):
        assert (C.nrows, C.ncols) == (a.nrows, b.ncols)
        assert_matches(C, oracle.spgemm(a, b), torch.float32, f"instance {i}")
        assert torch.equal(C.colptr, Q.colptr) and torch.equal(C.rowidx, Q.rowidx) and torch.equal(C.values, Q.values)
    with pytest.raises(ValueError):
        Bt.spgemm_batched([(dev[0][0], dev[-1][1])])
