"""GPU parity of the gradient path (transpose, masked X^T Y, permute,
autograd) against the CPU oracle's direct gradient formulas."""
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


def _forward(A, B):
    C, _ = S.Engine(A.to("cuda"), B.to("cuda"), 1).run()
    return C


def _targets(C, seed=9):
    col = torch.repeat_interleave(torch.arange(C.ncols, device=C.colptr.device), C.colptr[1:] - C.colptr[:-1])
    return synth.target_values(C.rowidx, col, C.ncols, seed, C.values.dtype), col


def _oracle_grads(A, B, C_dev, T_dev):
    """Oracle gradients for dC = C - T, with C and T taken from the oracle's
    own product and the coordinate-defined targets."""
    P = oracle.spgemm(A, B)
    col = np.repeat(np.arange(P.ncols), np.diff(P.colptr))
    T = synth.target_values(torch.from_numpy(P.rowidx.astype(np.int64)), torch.from_numpy(col), P.ncols, 9,
                            torch.float64).numpy()
    dC = oracle.Mat(P.nrows, P.ncols, P.colptr, P.rowidx, P.values - T)
    gA = oracle.grad_a(A, B, dC)
    gB = oracle.grad_b(A, B, dC)
    # scale of each gradient entry for the float32 bound: sum of |terms|
    adC = oracle.Mat(P.nrows, P.ncols, P.colptr, P.rowidx, np.abs(P.values - T) + P.absum)
    Aa = oracle.as_mat(A)
    Ba = oracle.as_mat(B)
    sA = oracle.grad_a(Aa, oracle.Mat(Ba.nrows, Ba.ncols, Ba.colptr, Ba.rowidx, np.abs(Ba.values)), adC)
    sB = oracle.grad_b(oracle.Mat(Aa.nrows, Aa.ncols, Aa.colptr, Aa.rowidx, np.abs(Aa.values)), Ba, adC)
    return gA, gB, sA, sB, P


def _check_grads(A, B, dtype, tol):
    Ad, Bd = A.to("cuda"), B.to("cuda")
    C = _forward(A, B)
    T, _ = _targets(C)
    dC = (C.values - T.to(C.values.dtype)).contiguous()
    bw = S.Backward(Ad, Bd, C)
    dA, dB = bw(dC)
    bw.check()
    gA, gB, sA, sB, P = _oracle_grads(A, B, C, T)
    dA, dB = dA.double().cpu().numpy(), dB.double().cpu().numpy()
    assert np.all(np.abs(dA - gA) <= tol * sA + 1e-300), float(np.max(np.abs(dA - gA) / np.maximum(sA, 1e-300)))
    assert np.all(np.abs(dB - gB) <= tol * sB + 1e-300), float(np.max(np.abs(dB - gB) / np.maximum(sB, 1e-300)))
    return dA, dB, C, dC


def test_transpose_matches_definition():
    print("case: transpose", flush=True)
    A = synth.shuffle_within_columns(synth.rmat(12, 8, 3, dtype=torch.float32), 1)
    Ad = A.to("cuda")
    T, perm = S.transpose(Ad)
    cp, ri, v = host_sorted(T)
    # reference: the (row, col) pairs swapped, grouped by the new column
    col = np.repeat(np.arange(A.ncols), np.diff(A.colptr.numpy()))
    rows = A.rowidx.numpy()
    order = np.lexsort((col, rows))
    assert np.array_equal(cp, np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=A.nrows))]))
    assert np.array_equal(ri, col[order])
    assert np.array_equal(v.astype(np.float32), A.values.numpy()[order])
    assert torch.equal(T.values, Ad.values[perm])


def test_permute_gather_scatter():
    print("case: permute", flush=True)
    x = torch.randn(100003, dtype=torch.float64, device="cuda")
    p = torch.randperm(100003, device="cuda")
    g = S.permute(x, p, False)
    assert torch.equal(g, x[p])
    s = S.permute(x, p, True)
    ref = torch.empty_like(x)
    ref[p] = x
    assert torch.equal(s, ref)


@pytest.mark.parametrize("min_bin", [0, 2, 4, 5])
def test_masked_xty_vs_oracle(min_bin):
    print(f"case: masked_xty bin {min_bin}", flush=True)
    S._lib.spgemm_debug_min_bin(min_bin)
    X = synth.erdos_renyi(7000, 900, 40, 1, torch.float64, dist="normal")
    Y = synth.erdos_renyi(7000, 700, 300, 2, torch.float64, dist="normal")  # dense-ish columns of Y
    M = synth.erdos_renyi(900, 700, 70, 3, torch.float64)
    out = S.masked_xty(X.to("cuda"), Y.to("cuda"), M.to("cuda")).cpu().numpy()
    ref = oracle.masked_xty(X, Y, M)
    scale = oracle.masked_xty(X.with_values(X.values.abs()), Y.with_values(Y.values.abs()), M)
    assert np.all(np.abs(out - ref) <= 1e-12 * scale)


def test_masked_xty_heavy_long_columns():
    """Columns of Y beyond the largest LDS table and long X columns."""
    print("case: masked_xty heavy", flush=True)
    X = synth.erdos_renyi(20000, 300, 500, 5, torch.float32, dist="normal")
    Y = synth.erdos_renyi(20000, 40, 9000, 6, torch.float32, dist="normal")
    M = synth.erdos_renyi(300, 40, 100, 7, torch.float32)
    out = S.masked_xty(X.to("cuda"), Y.to("cuda"), M.to("cuda")).double().cpu().numpy()
    ref = oracle.masked_xty(X, Y, M)
    scale = oracle.masked_xty(X.with_values(X.values.abs()), Y.with_values(Y.values.abs()), M)
    assert np.all(np.abs(out - ref) <= 1e-5 * scale)


def test_grads_fp64_small():
    print("case: grads fp64", flush=True)
    A = synth.erdos_renyi(3000, 2500, 9, 11, torch.float64, dist="normal")
    B = synth.erdos_renyi(2500, 2000, 7, 12, torch.float64, dist="normal")
    _check_grads(A, B, torch.float64, 1e-12)


def test_grads_fp32_er262k_shape_reduced():
    """Workload-4 structure (independent ER patterns, 16 per column, N(0,1))
    at n = 32768."""
    print("case: grads fp32 er32k", flush=True)
    A = synth.erdos_renyi(32768, 32768, 16, 21, torch.float32, dist="normal")
    B = synth.erdos_renyi(32768, 32768, 16, 22, torch.float32, dist="normal")
    dA, dB, C, dC = _check_grads(A, B, torch.float32, 1e-5)
    # <dA, A> = <dC, C> = <dB, B> (C is bilinear in A and B)
    dc = float((dC.double() * C.values.double()).sum())
    assert abs(float(dA @ A.values.double().numpy()) - dc) <= 1e-4 * abs(dc)
    assert abs(float(dB @ B.values.double().numpy()) - dc) <= 1e-4 * abs(dc)


def test_grads_rmat_heavy_fp32():
    """Skewed patterns: heavy columns of C (and of C^T) in the backward."""
    print("case: grads rmat", flush=True)
    A = synth.rmat(13, 16, 4, dtype=torch.float32)
    _check_grads(A, A, torch.float32, 1e-5)


def test_autograd_function_matches_oracle():
    print("case: autograd", flush=True)
    A = synth.erdos_renyi(4000, 3000, 12, 31, torch.float64, dist="normal")
    B = synth.erdos_renyi(3000, 3500, 10, 32, torch.float64, dist="normal")
    Ad, Bd = A.to("cuda"), B.to("cuda")
    a = Ad.values.clone().requires_grad_(True)
    b = Bd.values.clone().requires_grad_(True)
    cv, ccp, cri = S.SpGEMMFn.apply(a, b, Ad, Bd)
    C = S.CSC(A.nrows, B.ncols, ccp, cri, cv.detach())
    T, _ = _targets(C)
    loss = 0.5 * ((cv - T) ** 2).sum()
    loss.backward()
    gA, gB, sA, sB, P = _oracle_grads(A, B, C, T)
    assert np.all(np.abs(a.grad.cpu().numpy() - gA) <= 1e-12 * sA + 1e-300)
    assert np.all(np.abs(b.grad.cpu().numpy() - gB) <= 1e-12 * sB + 1e-300)


def test_finite_differences_fp64_n2048():
    """Central differences of the loss in float64 through the GPU forward,
    against the GPU gradient, on the n = 2048, 16-per-column instance."""
    print("case: fd", flush=True)
    n = 2048
    A = synth.erdos_renyi(n, n, 16, 101, torch.float64, dist="normal").to("cuda")
    B = synth.erdos_renyi(n, n, 16, 102, torch.float64, dist="normal").to("cuda")

    def loss(av, bv):
        C, _ = S.Engine(A.with_values(av), B.with_values(bv), 1).run()
        T, _ = _targets(C)
        return 0.5 * float(((C.values - T) ** 2).sum())

    C, _ = S.Engine(A, B, 1).run()
    T, _ = _targets(C)
    dA, dB = S.Backward(A, B, C)((C.values - T).contiguous())
    g = torch.Generator(device="cpu").manual_seed(0)
    h = 1e-5
    for _ in range(4):
        ua = torch.randn(A.nnz, generator=g, dtype=torch.float64).cuda()
        ub = torch.randn(B.nnz, generator=g, dtype=torch.float64).cuda()
        fd = (loss(A.values + h * ua, B.values + h * ub) - loss(A.values - h * ua, B.values - h * ub)) / (2 * h)
        an = float((dA * ua).sum() + (dB * ub).sum())
        assert abs(fd - an) <= 1e-6 * abs(an)
