"""A·Aᵀ, the paper's second workload (Sec. V: products of the Rice-kmers and
Metaclust matrices with their transposes; Sec. I: similarity and overlap
detection formed as A·Aᵀ in batches): the transpose on the GPU, then the
product, against the oracle's product with Aᵀ formed on the host by scipy."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import synth
from tests.gpu_util import assert_matches

pytestmark = pytest.mark.gpu

S = None


def setup_module(module):
    global S
    import paper_2010_08526_amd as lib
    S = lib


def _host_transpose(A):
    M = sp.csc_matrix((A.values.numpy(), A.rowidx.numpy(), A.colptr.numpy()), shape=(A.nrows, A.ncols))
    T = M.T.tocsc()
    return synth.CSC(A.ncols, A.nrows, torch.from_numpy(T.indptr.astype(np.int64)),
                     torch.from_numpy(T.indices.astype(np.int32)), torch.from_numpy(T.data))


@pytest.mark.parametrize("which,m,k", [("kmer-like cf~2", 20_000, 400_000), ("metaclust-like cf~1.1", 2_000_000, 400_000)])
@pytest.mark.parametrize("batches", [1, 3])
def test_aat_matches_oracle(which, m, k, batches):
    """Two entries per column of A at distinct uniform rows: with k >> m the
    diagonal collects most collisions (cf about 2), with m > k almost none."""
    print(f"case: aat {which} b={batches}", flush=True)
    A = synth.erdos_renyi(m, k, 2, 31, torch.float32)
    Ad = A.to("cuda")
    At, _ = S.transpose(Ad, perm=False)
    eng = S.Engine(Ad, At, 1, None)
    if batches > 1:
        plan = eng.plan()
        total_out = int((8 * plan.nnz_host[0] + 8).sum())
        eng.budget_bytes = (eng.input_bytes + eng.reserve_bytes + total_out // batches +
                            int(plan.nnz_host[0].max()) * 8 + 8)
    C, plan = eng.run()
    torch.cuda.synchronize()
    assert plan.nbatches >= batches
    P = oracle.spgemm(A, _host_transpose(A))
    cf = 4 * k / P.nnz
    assert (1.8 < cf < 2.1) if m < k else (1.05 < cf < 1.15), cf
    assert_matches(C, P, torch.float32, which)
