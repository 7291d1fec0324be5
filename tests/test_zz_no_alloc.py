"""The allocation-free batched forward (a fixed per-device scratch array
inside the library instead of a workspace argument) against the workspace
form of the same entry point and the oracle, on two calls in a row, the
second on a smaller input."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import assert_matches, host_sorted

pytestmark = pytest.mark.gpu


def _outputs(nnz_cap, n, vdt):
    return (torch.empty(n, dtype=torch.int64, device="cuda"), torch.empty(n, dtype=torch.int64, device="cuda"),
            torch.empty(n + 1, dtype=torch.int64, device="cuda"),
            torch.full((max(1, nnz_cap),), -1, dtype=torch.int32, device="cuda"),
            torch.full((max(1, nnz_cap),), float("nan"), dtype=vdt, device="cuda"))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_forward_matches_workspace_forward(dtype):
    import paper_2010_08526_amd as S
    import paper_2010_08526_amd.batched as Bt
    cases = [(24, 61, 4096), (7, 62, 1500)]  # (instances, seed, largest n_i): the second call is smaller
    for count, seed, nmax in cases:
        print(f"case: noalloc forward {dtype} count={count} seed={seed}", flush=True)
        spec = synth.batch_spec(count, seed, nmin=64, nmax=nmax)
        A, B, off = synth.batch_packed(spec, seed, dtype, "cuda")
        assert S.workspace_size(S.OP_BATCHED_FORWARD, A, B, 0, B.ncols) <= Bt.NOALLOC_SCRATCH_BYTES
        eng = Bt.BatchedEngine(A, B)  # the workspace form
        eng.forward()
        eng.check()
        ref = host_sorted(eng.C)
        n = B.ncols
        flops, nnz, cp, ri, v = _outputs(eng.nnz_c, n, dtype)
        Bt.batched_forward_noalloc(A, B, eng.nnz_c, flops, nnz, cp, ri, v)
        torch.cuda.synchronize()
        assert torch.equal(flops, eng.flops) and torch.equal(nnz, eng.nnz)
        assert int(cp[-1]) == eng.nnz_c
        C = S.CSC(A.nrows, n, cp, ri[:eng.nnz_c], v[:eng.nnz_c])
        got = host_sorted(C)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        P = oracle.spgemm(A.to("cpu"), B.to("cpu"))
        assert_matches(C, P, dtype, f"noalloc count={count}")
        assert_matches(eng.C, P, dtype, f"workspace form count={count}")
