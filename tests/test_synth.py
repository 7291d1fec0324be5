"""Pins of the seeded input generators."""
from __future__ import annotations

import numpy as np
import torch

import synth
from synth.rng import GOLDEN, Stream, mix64


def test_splitmix64_published_outputs():
    """SplitMix64 seeded with 0 starts 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    0x06c45d188009454f (the reference sequence of Steele et al.'s generator)."""
    z = torch.tensor([1, 2, 3], dtype=torch.int64) * GOLDEN  # wraps mod 2^64
    got = [x & ((1 << 64) - 1) for x in mix64(z).tolist()]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_stream_uniform_and_randint_ranges():
    s = Stream(1, 2)
    idx = torch.arange(200000)
    u = s.uniform(idx)
    assert float(u.min()) >= 0.0 and float(u.max()) < 1.0
    assert abs(float(u.mean()) - 0.5) < 0.005
    r = s.randint(idx, 7)
    assert int(r.min()) == 0 and int(r.max()) == 6
    counts = torch.bincount(r, minlength=7).double()
    assert float((counts / counts.sum() - 1 / 7).abs().max()) < 0.01
    z = s.normal(idx)
    assert abs(float(z.mean())) < 0.01 and abs(float(z.std()) - 1) < 0.01


def test_erdos_renyi_exact_degree_distinct_rows():
    A = synth.erdos_renyi(300, 500, 9, 3)
    cp = A.colptr.numpy()
    assert np.all(np.diff(cp) == 9)
    ri = A.rowidx.numpy()
    assert ri.min() >= 0 and ri.max() < 300
    for j in range(A.ncols):
        assert len(set(ri[cp[j]:cp[j + 1]].tolist())) == 9
    v = A.values.numpy()
    assert v.min() > 0 and v.max() <= 1.0
    # Floyd's algorithm gives uniform subsets: every row about equally likely
    B = synth.erdos_renyi(300, 20000, 9, 5)
    cnt = np.bincount(B.rowidx.numpy(), minlength=300)
    chi2 = float(((cnt - cnt.mean()) ** 2 / cnt.mean()).sum())  # ~ chi-square, 299 dof
    assert chi2 < 299 + 6 * np.sqrt(2 * 299)


def test_er_full_degree_is_full_column():
    A = synth.erdos_renyi(16, 10, 16, 4)
    ri = A.rowidx.numpy().reshape(10, 16)
    assert all(sorted(r.tolist()) == list(range(16)) for r in ri)


def test_rmat_symmetric_dedup():
    A = synth.rmat(10, 16, 9, dtype=torch.float32)
    n = A.ncols
    cp, ri = A.colptr.numpy(), A.rowidx.numpy()
    D = np.zeros((n, n), bool)
    col = np.repeat(np.arange(n), np.diff(cp))
    D[ri, col] = True
    assert np.array_equal(D, D.T)
    assert D.sum() == A.nnz  # no duplicates
    deg = np.diff(cp)
    assert deg[:8].mean() > 10 * deg.mean()  # hubs at low ids
    v = A.values.numpy()
    assert v.dtype == np.float32 and v.min() > 0 and v.max() <= 1.0


def test_protein_like_properties():
    A = synth.protein_like(20000, 7)
    n = A.ncols
    cp, ri = A.colptr.numpy(), A.rowidx.numpy()
    col = np.repeat(np.arange(n), np.diff(cp))
    assert not np.any(ri == col)  # no self loops
    keys = set(zip(ri.tolist(), col.tolist()))
    assert all((c, r) in keys for r, c in list(keys)[:5000])
    s = np.zeros(n)
    np.add.at(s, col, A.values.numpy().astype(np.float64))
    nz = np.diff(cp) > 0
    assert np.allclose(s[nz], 1.0, atol=1e-5)
    deg = np.diff(cp)
    assert 30 < deg.mean() < 60
    assert abs(synth.matrices._powerlaw_mean(synth.powerlaw_xmin(2.1, 50, 5000), 2.1, 5000) - 50) < 1e-9


def test_generators_deterministic():
    a = synth.rmat(9, 8, 1)
    b = synth.rmat(9, 8, 1)
    assert torch.equal(a.rowidx, b.rowidx) and torch.equal(a.values, b.values)
    c = synth.rmat(9, 8, 2)
    assert not torch.equal(a.rowidx, c.rowidx) or not torch.equal(a.values, c.values)


def test_batch_spec_ranges():
    spec = synth.batch_spec(4096, 5)
    assert int(spec.n.min()) >= 256 and int(spec.n.max()) <= 65536
    assert int(spec.dA.min()) >= 4 and int(spec.dA.max()) <= 32
    ln = torch.log(spec.n.double())
    assert abs(float(ln.mean()) - 0.5 * (np.log(256) + np.log(65536))) < 0.1


def test_targets_depend_on_coordinates_only():
    r = torch.tensor([3, 1, 4, 1])
    c = torch.tensor([0, 2, 2, 2])
    t = synth.target_values(r, c, 10, 8)
    assert t[1] == t[3] and t[0] != t[1]


def test_tie_heavy_columns_and_values():
    counts = [0, 1, 7, 50, 50, 3]
    M = synth.tie_heavy(50, counts, 4, torch.float64, levels=9, nan_frac=0.05)
    assert M.colptr.tolist() == np.cumsum([0] + counts).tolist()
    for j in range(M.ncols):
        r = M.rowidx[M.colptr[j]:M.colptr[j + 1]].numpy()
        assert r.size == np.unique(r).size and (r.size == 0 or (r.min() >= 0 and r.max() < 50))
    v = M.values.numpy()
    finite = v[~np.isnan(v)]
    assert set(np.unique(finite).tolist()) <= {-2.0 + 0.5 * i for i in range(9)}
    # deterministic, and a full column is a permutation of the rows
    M2 = synth.tie_heavy(50, counts, 4, torch.float64, levels=9, nan_frac=0.05)
    assert torch.equal(M.rowidx, M2.rowidx) and np.array_equal(v.view(np.uint64), M2.values.numpy().view(np.uint64))
    assert sorted(M.rowidx[M.colptr[3]:M.colptr[4]].tolist()) == list(range(50))
    # many entries: both zero signs and about the NaN fraction asked for
    B = synth.tie_heavy(1000, [1000] * 40, 5, torch.float32, levels=9, nan_frac=0.02)
    bv = B.values.numpy()
    zeros = bv[bv == 0]
    assert np.signbit(zeros).any() and (~np.signbit(zeros)).any()
    assert 0.015 < np.isnan(bv).mean() < 0.025
    # rows are not left sorted inside a column
    assert not all(np.all(np.diff(B.rowidx[B.colptr[j]:B.colptr[j + 1]].numpy()) > 0) for j in range(3))
