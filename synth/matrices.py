"""Seeded synthetic sparse matrices in CSC form.

Every generator here is a pure function of its arguments: the same call
gives the same bytes on the CPU and on a GPU (see ``synth.rng``).  Storage
is CSC with int64 column pointers, int32 row indices (rows unique within a
column, in generation order, i.e. not necessarily sorted) and float32 or
float64 values.

The families follow the workloads the paper evaluates on (protein
similarity graphs, a power-law social graph) and the shapes used to
exercise the one-GPU path: fixed-degree Erdos-Renyi, R-MAT, a Chung-Lu
power-law graph with column-stochastic values, and a batch of uneven
Erdos-Renyi pairs.  The module holds no SpGEMM arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .rng import Stream

# Stream tags: one per kind of draw so that no two quantities share counters.
TAG_ROWS, TAG_VALS, TAG_RMAT, TAG_WEIGHT, TAG_EDGE, TAG_TARGET, TAG_SHUFFLE, TAG_BATCH = range(1, 9)
TAG_PRUNE_ROWS, TAG_PRUNE_VALS = 9, 10


@dataclass
class CSC:
    """A CSC matrix held in torch tensors (any device)."""

    nrows: int
    ncols: int
    colptr: torch.Tensor  # int64 [ncols + 1]
    rowidx: torch.Tensor  # int32 [nnz]
    values: torch.Tensor | None  # float32 / float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    @property
    def device(self) -> torch.device:
        return self.rowidx.device

    def to(self, device) -> "CSC":
        v = None if self.values is None else self.values.to(device)
        return CSC(self.nrows, self.ncols, self.colptr.to(device), self.rowidx.to(device), v)

    def with_values(self, values: torch.Tensor | None) -> "CSC":
        return CSC(self.nrows, self.ncols, self.colptr, self.rowidx, values)

    def col_index(self) -> torch.Tensor:
        """Column id of every stored entry (int64 [nnz])."""
        counts = self.colptr[1:] - self.colptr[:-1]
        return torch.repeat_interleave(torch.arange(self.ncols, device=self.colptr.device), counts)


def _colptr_from_counts(counts: torch.Tensor) -> torch.Tensor:
    cp = torch.zeros(counts.numel() + 1, dtype=torch.int64, device=counts.device)
    cp[1:] = torch.cumsum(counts.to(torch.int64), 0)
    return cp


def _values(seed: int, n: int, dtype: torch.dtype, device, dist: str, tag: int = TAG_VALS,
            offset: int = 0) -> torch.Tensor:
    s = Stream(seed, tag)
    idx = torch.arange(offset, offset + n, device=device, dtype=torch.int64)
    if dist == "uniform":  # (0, 1]: never an exact zero
        v = 1.0 - s.uniform(idx)
    elif dist == "normal":
        v = s.normal(idx)
    else:
        raise ValueError(dist)
    return v.to(dtype)


def _floyd_rows(seed: int, m: torch.Tensor, d: torch.Tensor, dmax: int, counter_base: torch.Tensor,
                tag: int = TAG_ROWS) -> torch.Tensor:
    """Distinct uniform rows per column by Floyd's sampling algorithm
    (Bentley and Floyd, CACM 30(9), 1987), run for all columns at once.

    m, d, counter_base: int64 [ncols] (rows in the column's matrix, rows to
    draw, first counter of the column).  Returns int64 [ncols, dmax]; slots
    t >= d[col] hold -1.
    """
    s = Stream(seed, tag)
    ncols = m.numel()
    rows = torch.full((ncols, dmax), -1, dtype=torch.int64, device=m.device)
    for t in range(dmax):
        active = t < d
        hi = m - d + t  # Floyd: for J = m-d+t, draw T in [0, J]; take J if T is taken
        hi = torch.where(active, hi, torch.zeros_like(hi))
        r = s.randint(counter_base + t, hi + 1)
        if t:
            dup = (rows[:, :t] == r[:, None]).any(1)
            r = torch.where(dup, hi, r)
        rows[:, t] = torch.where(active, r, torch.full_like(r, -1))
    return rows


def erdos_renyi(m: int, n: int, d: int, seed: int, dtype=torch.float64, device="cpu",
                dist: str = "uniform") -> CSC:
    """m x n matrix with exactly d entries per column at distinct uniform rows."""
    if d > m:
        raise ValueError("degree exceeds rows")
    dev = torch.device(device)
    cols = torch.arange(n, device=dev, dtype=torch.int64)
    if d == 0:
        return CSC(m, n, torch.zeros(n + 1, dtype=torch.int64, device=dev),
                   torch.zeros(0, dtype=torch.int32, device=dev), torch.zeros(0, dtype=dtype, device=dev))
    rows = _floyd_rows(seed, torch.full((n,), m, dtype=torch.int64, device=dev),
                       torch.full((n,), d, dtype=torch.int64, device=dev), d, cols * d)
    rowidx = rows.reshape(-1).to(torch.int32)
    colptr = torch.arange(n + 1, device=dev, dtype=torch.int64) * d
    vals = _values(seed, n * d, dtype, dev, dist)
    return CSC(m, n, colptr, rowidx, vals)


def _pairs_to_csc(r: torch.Tensor, c: torch.Tensor, n: int, m: int, seed: int, dtype, dist="uniform") -> CSC:
    """Deduplicate (row, col) pairs into a CSC with rows sorted per column,
    values drawn per stored entry."""
    keys = torch.unique(c * m + r)  # sorted: by column, then row
    col = keys // m
    row = keys - col * m
    counts = torch.bincount(col, minlength=n)
    vals = _values(seed, keys.numel(), dtype, keys.device, dist)
    return CSC(m, n, _colptr_from_counts(counts), row.to(torch.int32), vals)


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, dtype=torch.float32,
         device="cpu", symmetrize=True, chunk: int = 1 << 23) -> CSC:
    """R-MAT graph (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of
    edge_factor * 2**scale edges picks a quadrant per level with
    probabilities (a, b, c, 1-a-b-c).  No noise and no vertex permutation,
    so hubs sit at low ids.  Self-loops are kept.  With ``symmetrize`` the
    pattern is A | A^T; duplicates are removed; values 1-U[0,1) per stored
    entry."""
    dev = torch.device(device)
    n = 1 << scale
    ne = edge_factor * n
    s = Stream(seed, TAG_RMAT)
    rs, cs = [], []
    for e0 in range(0, ne, chunk):
        e = torch.arange(e0, min(ne, e0 + chunk), device=dev, dtype=torch.int64)
        r = torch.zeros_like(e)
        cc = torch.zeros_like(e)
        for lvl in range(scale):
            u = s.uniform(e * scale + lvl)
            rbit = (u >= a + b).to(torch.int64)  # quadrants c, d: lower half
            cbit = (((u >= a) & (u < a + b)) | (u >= a + b + c)).to(torch.int64)  # quadrants b, d
            r = (r << 1) | rbit
            cc = (cc << 1) | cbit
        rs.append(r)
        cs.append(cc)
    r = torch.cat(rs)
    cc = torch.cat(cs)
    if symmetrize:
        r, cc = torch.cat([r, cc]), torch.cat([cc, r])
    return _pairs_to_csc(r, cc, n, n, seed, dtype)


def _powerlaw_mean(xmin: float, gamma: float, cap: float) -> float:
    g1, g2 = 1.0 - gamma, 2.0 - gamma
    return (g1 / g2) * (cap ** g2 - xmin ** g2) / (cap ** g1 - xmin ** g1)


def powerlaw_xmin(gamma: float, mean: float, cap: float) -> float:
    """Lower cut-off of a power law x^-gamma on [xmin, cap] with the given mean
    (bisection; the mean grows with xmin)."""
    lo, hi = 1e-6, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _powerlaw_mean(mid, gamma, cap) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def protein_like(n: int, seed: int, gamma=2.1, mean=50.0, cap=5000.0, dtype=torch.float32,
                 device="cpu", chunk: int = 1 << 24) -> CSC:
    """Chung-Lu graph (Chung and Lu, PNAS 2002) with expected degrees drawn
    from a power law x^-gamma truncated to [xmin, cap], xmin set so the mean
    is ``mean``.  About sum(w)/2 edges are drawn with both endpoints chosen
    with probability proportional to w; the pattern is symmetric with no
    self-loops and no duplicates.  Values 1-U[0,1), then each column is
    divided by its sum in float64 (column-stochastic), then rounded."""
    dev = torch.device(device)
    xmin = powerlaw_xmin(gamma, mean, cap)
    g1 = 1.0 - gamma
    sw = Stream(seed, TAG_WEIGHT)
    u = sw.uniform(torch.arange(n, device=dev, dtype=torch.int64))
    w = (xmin ** g1 - u * (xmin ** g1 - cap ** g1)) ** (1.0 / g1)  # inverse CDF
    cdf = torch.cumsum(w, 0)
    total = float(cdf[-1])
    cdf = cdf / total
    ne = int(round(total / 2))
    se = Stream(seed, TAG_EDGE)
    rs, cs = [], []
    for e0 in range(0, ne, chunk):
        e = torch.arange(e0, min(ne, e0 + chunk), device=dev, dtype=torch.int64)
        i = torch.searchsorted(cdf, se.uniform(2 * e), right=True).clamp_(max=n - 1)
        j = torch.searchsorted(cdf, se.uniform(2 * e + 1), right=True).clamp_(max=n - 1)
        keep = i != j
        rs.append(i[keep])
        cs.append(j[keep])
    r = torch.cat(rs)
    c = torch.cat(cs)
    A = _pairs_to_csc(torch.cat([r, c]), torch.cat([c, r]), n, n, seed, torch.float64)
    colsum = torch.zeros(n, dtype=torch.float64, device=dev)
    colsum.index_add_(0, A.col_index(), A.values)
    vals = A.values / colsum[A.col_index()]
    return A.with_values(vals.to(dtype))


def shuffle_within_columns(A: CSC, seed: int) -> CSC:
    """Random order of the entries inside every column (same entry set)."""
    key = Stream(seed, TAG_SHUFFLE).uniform(torch.arange(A.nnz, device=A.device))
    col = A.col_index().to(torch.float64)
    perm = torch.argsort(col + key * 0.5)  # keys in [0, 0.5) keep columns apart
    v = None if A.values is None else A.values[perm]
    return CSC(A.nrows, A.ncols, A.colptr.clone(), A.rowidx[perm].contiguous(), v)


def target_values(rows: torch.Tensor, cols: torch.Tensor, ncols: int, seed: int,
                  dtype=torch.float64) -> torch.Tensor:
    """Loss targets T(i, j) ~ N(0, 1) as a function of the coordinate (i, j),
    not of a storage slot, so any output order sees the same targets."""
    idx = rows.to(torch.int64) * ncols + cols.to(torch.int64)
    return Stream(seed, TAG_TARGET).normal(idx).to(dtype)


@dataclass
class BatchSpec:
    """Sizes of one batch of independent products C_i = A_i B_i."""

    n: torch.Tensor  # int64 [count]: A_i, B_i are n_i x n_i
    dA: torch.Tensor  # int64 [count]: entries per column of A_i
    dB: torch.Tensor  # int64 [count]


def batch_spec(count: int, seed: int, nmin=256, nmax=65536, dmin=4, dmax=32) -> BatchSpec:
    """n_i = round(exp(U[ln nmin, ln nmax])) (log-uniform), degrees uniform
    integers in [dmin, dmax], all per instance."""
    s = Stream(seed, TAG_BATCH)
    i = torch.arange(count, dtype=torch.int64)
    u = s.uniform(3 * i)
    n = torch.round(torch.exp(math.log(nmin) + u * (math.log(nmax) - math.log(nmin)))).to(torch.int64)
    dA = dmin + s.randint(3 * i + 1, dmax - dmin + 1)
    dB = dmin + s.randint(3 * i + 2, dmax - dmin + 1)
    return BatchSpec(n, dA, dB)


def batch_instance(spec: BatchSpec, i: int, seed: int, dtype=torch.float32, device="cpu") -> tuple[CSC, CSC]:
    """Instance i of a batch: independent Erdos-Renyi A_i and B_i."""
    n = int(spec.n[i])
    sa = seed * 1_000_003 + 2 * i + 1
    sb = seed * 1_000_003 + 2 * i + 2
    return (erdos_renyi(n, n, int(spec.dA[i]), sa, dtype, device),
            erdos_renyi(n, n, int(spec.dB[i]), sb, dtype, device))


def batch_packed(spec: BatchSpec, seed: int, dtype=torch.float32, device="cpu", first: int = 0,
                 count: int | None = None, chunk_cols: int = 1 << 22):
    """Instances [first, first+count) of a batch as two block-diagonal CSC
    matrices: instance i's A_i (n_i x n_i, dA_i distinct uniform rows per
    column) occupies rows and columns [o_i, o_i + n_i) of A, and likewise B_i
    in B, with o_i = n_first + ... + n_{i-1}.  Values 1-U[0,1).  Every draw is
    keyed by the instance's global column id, so an instance's bytes do not
    depend on which other instances are packed with it.

    Returns (A, B, offsets) with offsets int64 [count+1] (o_i and the total)."""
    dev = torch.device(device)
    count = spec.n.numel() - first if count is None else count
    n = spec.n[first:first + count].to(dev)
    off = torch.zeros(count + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(n, 0)
    total = int(off[-1])
    # global column id of each packed column: instance columns are numbered
    # across the whole batch (not just this slice)
    allcol = torch.zeros(spec.n.numel() + 1, dtype=torch.int64)
    allcol[1:] = torch.cumsum(spec.n, 0)
    gbase = int(allcol[first])
    inst = torch.repeat_interleave(torch.arange(count, device=dev), n)
    mats = []
    for which, degs, tag in ((0, spec.dA, 11), (1, spec.dB, 12)):
        d = degs[first:first + count].to(dev)[inst]  # per packed column
        m = n[inst]
        rows = torch.empty(0, dtype=torch.int32, device=dev)
        parts = []
        for c0 in range(0, total, chunk_cols):
            c1 = min(total, c0 + chunk_cols)
            gcol = torch.arange(c0, c1, device=dev, dtype=torch.int64) + gbase
            r = _floyd_rows(seed * 2 + which, m[c0:c1], d[c0:c1], 32, gcol * 32, tag=TAG_ROWS + 16 * tag)
            r = r + off[inst[c0:c1]][:, None]
            parts.append(r[r >= off[inst[c0:c1]][:, None]].to(torch.int32))  # drop the -1 padding
        rows = torch.cat(parts) if parts else rows
        cp = torch.zeros(total + 1, dtype=torch.int64, device=dev)
        cp[1:] = torch.cumsum(d, 0)
        # value of entry t of global column g: counter g * 32 + t
        gcol_e = torch.repeat_interleave(torch.arange(total, device=dev, dtype=torch.int64) + gbase, d)
        t = torch.arange(rows.numel(), device=dev, dtype=torch.int64) - cp[:-1].repeat_interleave(d)
        vals = (1.0 - Stream(seed * 2 + which, TAG_VALS + 16 * tag).uniform(gcol_e * 32 + t)).to(dtype)
        mats.append(CSC(total, total, cp, rows, vals))
    return mats[0], mats[1], off


def tie_heavy(m: int, counts, seed: int, dtype=torch.float32, levels: int = 9, nan_frac: float = 0.02,
              device="cpu", chunk: int = 1 << 24) -> CSC:
    """A matrix to prune: column j holds counts[j] distinct rows of [0, m) in
    random order (the first counts[j] of a random permutation), values drawn
    from ``levels`` equally spaced points of [-2, 2] (many ties), every zero
    with a random sign, NaN with probability ``nan_frac``."""
    dev = torch.device(device)
    counts = torch.as_tensor(counts, dtype=torch.int64)
    n = counts.numel()
    if n and int(counts.max()) > m:
        raise ValueError("count exceeds rows")
    sr, sv = Stream(seed, TAG_PRUNE_ROWS), Stream(seed, TAG_PRUNE_VALS)
    per = max(1, chunk // max(1, m))
    rows = []
    for c0 in range(0, n, per):
        c1 = min(n, c0 + per)
        idx = torch.arange(c0 * m, c1 * m, dtype=torch.int64).reshape(c1 - c0, m)
        perm = torch.argsort(sr.uniform(idx), dim=1)
        keep = torch.arange(m)[None, :] < counts[c0:c1, None]
        rows.append(perm[keep])
    rowidx = (torch.cat(rows) if rows else torch.zeros(0, dtype=torch.int64)).to(torch.int32)
    nnz = rowidx.numel()
    e = torch.arange(nnz, dtype=torch.int64)
    lvl = sv.randint(3 * e, levels).to(torch.float64)
    v = -2.0 + 4.0 * lvl / (levels - 1)
    v = torch.where((v == 0) & (sv.uniform(3 * e + 1) < 0.5), torch.full_like(v, -0.0), v)
    v = torch.where(sv.uniform(3 * e + 2) < nan_frac, torch.full_like(v, float("nan")), v)
    return CSC(m, n, _colptr_from_counts(counts), rowidx, v.to(dtype)).to(dev)
