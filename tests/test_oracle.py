"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against what the paper and mathematics fix:
hand-worked fixtures (tests/golden), numpy dense products, scipy's
independent sparse product, closed forms, invariants (Eq. 1, cf >= 1),
exact single-term products, permutation equivariance and brute force.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import Mat
from tests.helpers import csc_to_dense, dense_to_csc, pattern_dense, random_sparse, sort_columns

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _entries(P):
    out = {}
    for j in range(P.ncols):
        for p in range(P.colptr[j], P.colptr[j + 1]):
            out[(int(P.rowidx[p]), j)] = p
    return out


# ---------------------------------------------------------------- fixtures
def test_hand_worked_3x3():
    g = json.load(open(os.path.join(GOLDEN, "hand_3x3.json")))
    A = dense_to_csc(g["A_dense"])
    B = dense_to_csc(g["B_dense"])
    P = oracle.spgemm(A, B)
    assert P.nnz == g["nnz_C"]
    assert oracle.flops(A, B).tolist() == g["flops_per_col"]
    assert int(oracle.flops(A, B).sum()) == g["flops"]
    e = _entries(P)
    assert len(e) == len(g["C_entries"])
    for r, c, v, t in g["C_entries"]:
        p = e[(r, c)]
        assert P.values[p] == v
        assert P.terms[p] == t
    w = -(-A.ncols // g["layers"])
    for L, (cnt, ents) in enumerate(zip(g["layer_nnz_per_col"], g["layer_entries"])):
        D = oracle.spgemm(A, B, klo=L * w, khi=min(A.ncols, (L + 1) * w))
        assert np.diff(D.colptr).tolist() == cnt
        de = _entries(D)
        assert len(de) == len(ents)
        for r, c, v in ents:
            assert D.values[de[(r, c)]] == v


def test_hand_worked_cancellation_keeps_structural_zero():
    g = json.load(open(os.path.join(GOLDEN, "cancellation_1x1.json")))
    A = dense_to_csc(g["A_dense"])
    B = dense_to_csc(g["B_dense"])
    P = oracle.spgemm(A, B)
    assert P.nnz == g["nnz_C"] == 1
    assert P.values[0] == 0.0 and P.terms[0] == 2
    assert int(oracle.flops(A, B).sum()) == g["flops"]


# ------------------------------------------------------- numpy dense pins
@pytest.mark.parametrize("seed", range(12))
def test_tiny_random_vs_dense(seed):
    rng = np.random.default_rng(seed)
    m, k, n = (int(x) for x in rng.integers(1, 40, 3))
    dens = float(rng.choice([0.0, 0.02, 0.1, 0.3, 0.8]))
    A = random_sparse(m, k, dens, rng, dist="normal")
    B = random_sparse(k, n, float(rng.choice([0.05, 0.2, 0.5])), rng, dist="normal")
    P = oracle.spgemm(A, B)
    Ad, Bd = csc_to_dense(A), csc_to_dense(B)
    PA, PB = pattern_dense(A), pattern_dense(B)
    T = PA @ PB  # integer matmul: number of product terms per (i, j)
    assert np.array_equal(pattern_dense(P), (T > 0).astype(np.int64))
    Cd = csc_to_dense(P)
    ref = Ad @ Bd
    scale = np.abs(Ad) @ np.abs(Bd)
    assert np.all(np.abs(Cd - ref) <= 1e-14 * scale + 1e-300)
    assert np.array_equal(csc_to_dense(P, P.terms.astype(np.float64)), T.astype(np.float64))
    assert np.allclose(csc_to_dense(P, P.absum), scale, rtol=1e-14, atol=0)
    # flops = sum over (i,j) of term counts = sum_k nnz(A(:,k)) nnz(B(k,:))
    f = oracle.flops(A, B)
    assert f.sum() == T.sum() == (PA.sum(0) * PB.sum(1)).sum()
    assert np.array_equal(f, T.sum(0))
    # rows sorted per column, unique
    for j in range(P.ncols):
        r = P.rowidx[P.colptr[j]:P.colptr[j + 1]]
        assert np.all(np.diff(r) > 0)


def test_empty_and_degenerate():
    Z = Mat(5, 4, np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = dense_to_csc(np.eye(4))
    P = oracle.spgemm(Z, B)
    assert P.nnz == 0 and P.colptr.tolist() == [0] * 5
    A = dense_to_csc(np.arange(20, dtype=float).reshape(5, 4) % 3)
    P = oracle.spgemm(A, B, c0=2, c1=2)
    assert P.ncols == 0 and P.nnz == 0
    P = oracle.spgemm(A, B, klo=3, khi=3)  # empty layer
    assert P.nnz == 0
    E = Mat(4, 3, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))  # all-empty B
    assert oracle.spgemm(A, E).nnz == 0


# ----------------------------------------------------------- scipy pin
@pytest.mark.parametrize("seed", [0, 1])
def test_medium_vs_scipy(seed):
    from synth import erdos_renyi, rmat
    import torch
    if seed == 0:
        A = oracle.as_mat(erdos_renyi(10000, 10000, 6, 77, torch.float64))
        B = oracle.as_mat(erdos_renyi(10000, 8000, 5, 78, torch.float64))
    else:
        A = oracle.as_mat(rmat(13, 8, 5, dtype=torch.float64))
        B = A
    P = oracle.spgemm(A, B)
    SA = sp.csc_matrix((A.values, A.rowidx, A.colptr), shape=(A.nrows, A.ncols))
    SB = sp.csc_matrix((B.values, B.rowidx, B.colptr), shape=(B.nrows, B.ncols))
    S = (SA @ SB).tocsc()
    S.sort_indices()
    assert np.array_equal(S.indptr, P.colptr)  # positive values: scipy drops no entry
    assert np.array_equal(S.indices, P.rowidx)
    assert np.all(np.abs(S.data - P.values) <= 1e-14 * P.absum)


# --------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,da,db", [(4096, 8, 8), (2048, 16, 16), (1000, 3, 7)])
def test_flops_closed_form_er(n, da, db):
    from synth import erdos_renyi
    import torch
    A = erdos_renyi(n, n, da, 11, torch.float64)
    B = erdos_renyi(n, n, db, 12, torch.float64)
    f = oracle.flops(A, B)
    assert int(f.sum()) == n * da * db
    assert np.all(f == da * db)


def test_flops_symmetric_square_is_sum_of_squared_degrees():
    from synth import rmat
    import torch
    A = rmat(10, 8, 3, dtype=torch.float64)
    deg = np.diff(A.colptr.numpy())
    assert int(oracle.flops(A, A).sum()) == int((deg.astype(np.int64) ** 2).sum())


# ------------------------------------------------------------ invariants
@pytest.mark.parametrize("L", [1, 2, 3, 16, 40])
def test_eq1_chain_and_layer_merge(L):
    """flops >= sum_l nnz(D^l) >= nnz(C) (Eq. 1), and adding the partials by
    coordinate gives C (Merge, Sec. III-A)."""
    from synth import rmat
    import torch
    A = oracle.as_mat(rmat(9, 8, 21, dtype=torch.float64))
    P = oracle.spgemm(A, A)
    w = -(-A.ncols // L)
    tot = 0
    acc = {}
    for l in range(L):
        D = oracle.spgemm(A, A, klo=min(A.ncols, l * w), khi=min(A.ncols, (l + 1) * w))
        tot += D.nnz
        for (r, c), p in _entries(D).items():
            acc[(r, c)] = acc.get((r, c), 0.0) + D.values[p]
    fl = int(oracle.flops(A, A).sum())
    assert fl >= tot >= P.nnz
    assert P.nnz >= 1 and fl / P.nnz >= 1.0  # cf >= 1 (Sec. II-A)
    e = _entries(P)
    assert set(acc) == set(e)
    for key, p in e.items():
        assert abs(acc[key] - P.values[p]) <= 1e-13 * P.absum[p]
    if L == 1:
        assert tot == P.nnz


def test_column_ranges_concatenate():
    """Batches over output columns concatenate to C (Alg. 4, ColConcat)."""
    from synth import erdos_renyi
    import torch
    A = erdos_renyi(3000, 3000, 7, 5, torch.float64)
    P = oracle.spgemm(A, A)
    bounds = [0, 1, 700, 701, 2999, 3000]
    rows, vals = [], []
    for a, b in zip(bounds[:-1], bounds[1:]):
        Q = oracle.spgemm(A, A, c0=a, c1=b)
        assert np.array_equal(Q.colptr, P.colptr[a:b + 1] - P.colptr[a])
        rows.append(Q.rowidx)
        vals.append(Q.values)
    assert np.array_equal(np.concatenate(rows), P.rowidx)
    assert np.array_equal(np.concatenate(vals), P.values)


def test_single_term_products_are_exact():
    """Every entry of A*I, A*diag(s) and P*A is one product, hence the
    correctly rounded float64 product."""
    rng = np.random.default_rng(3)
    A = random_sparse(50, 40, 0.2, rng, dist="normal")
    Ad = csc_to_dense(A)
    P = oracle.spgemm(A, dense_to_csc(np.eye(40)))
    assert np.array_equal(csc_to_dense(P), Ad)
    s = rng.standard_normal(40)
    P = oracle.spgemm(A, dense_to_csc(np.diag(s)))
    assert np.array_equal(csc_to_dense(P), Ad * s[None, :])
    perm = rng.permutation(50)
    Pm = np.zeros((50, 50))
    Pm[np.arange(50), perm] = 1.0
    P = oracle.spgemm(dense_to_csc(Pm), A)
    assert np.array_equal(csc_to_dense(P), Ad[perm])
    assert np.all(P.terms == 1)


def test_permutation_equivariance():
    """(P A Q)(Q^T B R) = P (A B) R for permutation matrices P, Q, R."""
    rng = np.random.default_rng(9)
    A = random_sparse(30, 25, 0.15, rng)
    B = random_sparse(25, 35, 0.15, rng)
    Ad, Bd = csc_to_dense(A), csc_to_dense(B)
    p, q, r = rng.permutation(30), rng.permutation(25), rng.permutation(35)
    A2 = dense_to_csc(Ad[p][:, q])
    B2 = dense_to_csc(Bd[q][:, r])
    C = csc_to_dense(oracle.spgemm(A, B))
    C2 = csc_to_dense(oracle.spgemm(A2, B2))
    assert np.allclose(C2, C[p][:, r], rtol=1e-14, atol=0)
    assert np.array_equal(C2 != 0, (C != 0)[p][:, r])


def test_unsorted_inputs_give_same_product():
    """Hash SpGEMM needs no sorted input columns (Sec. IV-D): the product's
    entry set does not depend on the order inside input columns."""
    from synth import erdos_renyi, shuffle_within_columns
    import torch
    A = erdos_renyi(500, 500, 9, 4, torch.float64)
    As = shuffle_within_columns(A, 17)
    assert not torch.equal(A.rowidx, As.rowidx)
    P, Q = oracle.spgemm(A, A), oracle.spgemm(As, As)
    assert np.array_equal(P.colptr, Q.colptr) and np.array_equal(P.rowidx, Q.rowidx)
    assert np.all(np.abs(P.values - Q.values) <= 1e-14 * P.absum)


# ------------------------------------------------------------- backward
def _loss_parts(seed, m=20, k=15, n=18, dens=0.25):
    rng = np.random.default_rng(seed)
    A = random_sparse(m, k, dens, rng, dist="normal")
    B = random_sparse(k, n, dens, rng, dist="normal")
    P = oracle.spgemm(A, B)
    T = rng.standard_normal(P.nnz)
    dC = Mat(P.nrows, P.ncols, P.colptr, P.rowidx, P.values - T)
    return A, B, P, T, dC


@pytest.mark.parametrize("seed", range(6))
def test_gradients_vs_dense(seed):
    A, B, P, T, dC = _loss_parts(seed)
    G = csc_to_dense(dC)
    dA = oracle.grad_a(A, B, dC)
    dB = oracle.grad_b(A, B, dC)
    refA = (G @ csc_to_dense(B).T)
    refB = (csc_to_dense(A).T @ G)
    for j in range(A.ncols):
        for p in range(A.colptr[j], A.colptr[j + 1]):
            assert abs(dA[p] - refA[A.rowidx[p], j]) <= 1e-12 * (1 + abs(refA[A.rowidx[p], j]))
    for j in range(B.ncols):
        for p in range(B.colptr[j], B.colptr[j + 1]):
            assert abs(dB[p] - refB[B.rowidx[p], j]) <= 1e-12 * (1 + abs(refB[B.rowidx[p], j]))
    # C is bilinear in (A, B): <dA, A> = <dC, C> = <dB, B>
    dc = float(dC.values @ P.values)
    assert np.isclose(float(dA @ A.values), dc, rtol=1e-12, atol=1e-12)
    assert np.isclose(float(dB @ B.values), dc, rtol=1e-12, atol=1e-12)


def test_masked_xty_vs_dense():
    rng = np.random.default_rng(5)
    X = random_sparse(30, 12, 0.3, rng, dist="normal")
    Y = random_sparse(30, 14, 0.3, rng, dist="normal")
    M = random_sparse(12, 14, 0.4, rng)
    out = oracle.masked_xty(X, Y, M)
    ref = csc_to_dense(X).T @ csc_to_dense(Y)
    for j in range(M.ncols):
        for p in range(M.colptr[j], M.colptr[j + 1]):
            assert abs(out[p] - ref[M.rowidx[p], j]) <= 1e-13 * (1 + abs(ref[M.rowidx[p], j]))


def test_gradients_finite_differences():
    """Central differences of the loss 0.5 * sum over P(C) of (C - T)^2 in
    float64 on an n = 2048, 16-per-column instance.  Along any line the loss
    is a quartic, so the central difference error is h^2/6 * L'''."""
    from synth import erdos_renyi, target_values
    import torch
    n = 2048
    A = oracle.as_mat(erdos_renyi(n, n, 16, 101, torch.float64, dist="normal"))
    B = oracle.as_mat(erdos_renyi(n, n, 16, 102, torch.float64, dist="normal"))
    P = oracle.spgemm(A, B)
    col = np.repeat(np.arange(n), np.diff(P.colptr))
    T = target_values(torch.from_numpy(P.rowidx.astype(np.int64)), torch.from_numpy(col), n, 5).numpy()

    def loss(av, bv):
        Q = oracle.spgemm(Mat(n, n, A.colptr, A.rowidx, av), Mat(n, n, B.colptr, B.rowidx, bv))
        return 0.5 * float(((Q.values - T) ** 2).sum())

    dC = Mat(n, n, P.colptr, P.rowidx, P.values - T)
    dA = oracle.grad_a(A, B, dC)
    dB = oracle.grad_b(A, B, dC)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(4):
        ua = rng.standard_normal(A.nnz)
        ub = rng.standard_normal(B.nnz)
        fd = (loss(A.values + h * ua, B.values + h * ub) - loss(A.values - h * ua, B.values - h * ub)) / (2 * h)
        an = float(dA @ ua + dB @ ub)
        assert abs(fd - an) <= 1e-6 * abs(an)
    for q in rng.integers(0, A.nnz, 4):
        e = np.zeros(A.nnz)
        e[q] = 1.0
        fd = (loss(A.values + h * e, B.values) - loss(A.values - h * e, B.values)) / (2 * h)
        assert abs(fd - dA[q]) <= 1e-6 * max(1.0, abs(dA[q]))


# ---------------------------------------------------------------- planner
def _brute_best(col_bytes, avail):
    """Fewest contiguous batches that fit, then the smallest largest batch
    (dynamic programming over all split points)."""
    n = len(col_bytes)
    pre = np.concatenate([[0], np.cumsum(col_bytes)])
    INF = (10 ** 18, 10 ** 18)
    best = [INF] * (n + 1)  # (batches, max load) for prefix of length i
    best[0] = (0, 0)
    for i in range(1, n + 1):
        for s in range(i):
            load = int(pre[i] - pre[s])
            if load > avail or best[s] == INF:
                continue
            cand = (best[s][0] + 1, max(best[s][1], load))
            best[i] = min(best[i], cand)
    return best[n]


@pytest.mark.parametrize("seed", range(30))
def test_planner_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 14))
    cb = rng.integers(1, 50, n).tolist()
    avail = int(rng.integers(max(cb), 2 * sum(cb) + 1))
    bounds = oracle.plan_batches(cb, avail)
    loads = [sum(cb[a:b]) for a, b in zip(bounds[:-1], bounds[1:])]
    assert bounds[0] == 0 and bounds[-1] == n and all(x <= y for x, y in zip(bounds, bounds[1:]))
    assert all(x <= avail for x in loads)
    assert (len(loads), max(loads)) == _brute_best(cb, avail)
    assert len(loads) >= -(-sum(cb) // avail)  # Eq. (2) lower bound
    assert (len(loads) == 1) == (sum(cb) <= avail)


def test_planner_errors_and_monotone():
    with pytest.raises(ValueError):
        oracle.plan_batches([5, 6], 0)
    with pytest.raises(ValueError):
        oracle.plan_batches([5, 60], 50)
    cb = list(np.random.default_rng(1).integers(1, 100, 200))
    prev = None
    for avail in range(100, 20000, 377):
        b = len(oracle.plan_batches(cb, avail)) - 1
        if prev is not None:
            assert b <= prev
        prev = b


# ------------------------------------------------- per-column pruning of a batch
def _prune_fixture():
    with open(os.path.join(GOLDEN, "prune_topk_hand.json")) as f:
        g = json.load(f)
    cols = g["columns"]
    colptr = np.cumsum([0] + [len(c) for c in cols]).astype(np.int64)
    rows = np.array([e[0] for c in cols for e in c], np.int32)
    vals = np.array([np.nan if e[1] is None else e[1] for c in cols for e in c], np.float64)
    return g, Mat(g["nrows"], len(cols), colptr, rows, vals)


def test_prune_hand_worked():
    g, M = _prune_fixture()
    for case in g["cases"]:
        P = oracle.prune_topk(M, case["threshold"], case["k"])
        for j, exp in enumerate(case["expect"]):
            s, e = P.colptr[j], P.colptr[j + 1]
            got = list(zip(P.rowidx[s:e].tolist(), P.values[s:e].tolist()))
            assert [(r, v) for r, v in got] == [(r, v) for r, v in exp], (case, j)
            # the sign of a kept zero is the input's
            assert [np.signbit(v) for _, v in got] == [np.signbit(v) for _, v in exp], (case, j)


def _tie_heavy(seed, m=9, n=12, dens=0.6):
    """Random CSC with rows shuffled inside columns and values drawn from a
    small set (many ties, both signed zeros, NaN)."""
    rng = np.random.default_rng(seed)
    pool = np.array([-2.0, -1.0, -0.0, 0.0, 0.5, 1.0, 1.0, 2.0, np.nan])
    colptr, rows, vals = [0], [], []
    for _ in range(n):
        r = rng.permutation(m)[: rng.binomial(m, dens)]
        rows += r.tolist()
        vals += rng.choice(pool, r.size).tolist()
        colptr.append(len(rows))
    return Mat(m, n, np.array(colptr, np.int64), np.array(rows, np.int32), np.array(vals, np.float64))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("threshold,k", [(-5.0, 1), (-5.0, 3), (0.0, 2), (0.5, 0), (-0.5, 4), (-5.0, -1), (1.0, -1)])
def test_prune_brute_force(seed, threshold, k):
    """Characterisation independent of any sort: the kept set of a column is
    the unique subset of the candidates of size min(k, #candidates) in which
    every kept entry outranks every dropped candidate (greater value, or an
    equal value and a smaller row); kept entries keep their input order and
    values bit for bit."""
    M = _tie_heavy(seed)
    P = oracle.prune_topk(M, threshold, k)

    def outranks(a, b):  # (row, value) pairs
        return a[1] > b[1] or (a[1] == b[1] and a[0] < b[0])

    for j in range(M.ncols):
        s, e = M.colptr[j], M.colptr[j + 1]
        col = [(int(r), float(v), p) for p, (r, v) in enumerate(zip(M.rowidx[s:e], M.values[s:e]))]
        cand = [c for c in col if c[1] >= threshold]
        want = len(cand) if k < 0 else min(k, len(cand))
        ps, pe = P.colptr[j], P.colptr[j + 1]
        kept_rows = P.rowidx[ps:pe].tolist()
        assert len(kept_rows) == want
        kept = [c for c in cand if c[0] in kept_rows]
        dropped = [c for c in cand if c[0] not in kept_rows]
        assert len(kept) == want
        assert all(outranks(a, b) for a in kept for b in dropped)
        assert kept_rows == [c[0] for c in kept]  # input order
        assert np.array_equal(P.values[ps:pe].view(np.uint64), np.array([c[1] for c in kept]).view(np.uint64))


def test_prune_special_cases():
    M = _tie_heavy(11, m=30, n=20)
    finite = ~np.isnan(M.values)
    # no threshold and no limit: the matrix minus its NaN entries
    P = oracle.prune_topk(M, -np.inf, -1)
    assert P.nnz == int(finite.sum()) and np.array_equal(P.rowidx, M.rowidx[finite])
    # a limit no column reaches is the threshold alone, a plain mask
    for t in (-1.0, 0.0, 1.0):
        P = oracle.prune_topk(M, t, 10 ** 6)
        keep = M.values >= t
        assert np.array_equal(P.rowidx, M.rowidx[keep]) and np.array_equal(P.values, M.values[keep])
        assert np.diff(P.colptr).tolist() == [int(keep[M.colptr[j]:M.colptr[j + 1]].sum()) for j in range(M.ncols)]
    # nothing kept
    assert oracle.prune_topk(M, -np.inf, 0).nnz == 0 and oracle.prune_topk(M, np.inf, -1).nnz == 0
    # k = 1 on distinct values is the column maximum (np.argmax)
    rng = np.random.default_rng(3)
    R = random_sparse(40, 25, 0.3, rng)
    P = oracle.prune_topk(R, -np.inf, 1)
    for j in range(R.ncols):
        s, e = R.colptr[j], R.colptr[j + 1]
        if e > s:
            assert P.colptr[j + 1] - P.colptr[j] == 1
            assert P.values[P.colptr[j]] == R.values[s:e].max() and P.rowidx[P.colptr[j]] == R.rowidx[s + np.argmax(R.values[s:e])]
    # an empty matrix and a matrix without columns
    E = Mat(5, 3, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert oracle.prune_topk(E, 0.0, 2).colptr.tolist() == [0, 0, 0, 0]
    assert oracle.prune_topk(Mat(5, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)), 0.0, 2).nnz == 0


def test_aat_closed_forms():
    """A A^T (the paper's second workload shape): symmetric, its diagonal the
    row sums of squares, equal to scipy's product; cf near 2 for two entries
    per column with k >> m."""
    rng = np.random.default_rng(8)
    m, k = 300, 20000
    rows = np.stack([rng.choice(m, 2, replace=False) for _ in range(k)]).reshape(-1).astype(np.int32)
    vals = rng.random(2 * k) + 0.5
    A = Mat(m, k, np.arange(0, 2 * k + 1, 2, dtype=np.int64), rows, vals)
    S_ = sp.csc_matrix((vals, rows, A.colptr), shape=(m, k))
    T = S_.T.tocsc()
    At = Mat(k, m, T.indptr.astype(np.int64), T.indices.astype(np.int32), T.data.astype(np.float64))
    P = oracle.spgemm(A, At)
    D = np.zeros((m, m))
    for j in range(m):
        for p in range(P.colptr[j], P.colptr[j + 1]):
            D[P.rowidx[p], j] = P.values[p]
    assert np.allclose(D, D.T, rtol=1e-13, atol=0)
    assert np.allclose(np.diag(D), np.asarray(S_.multiply(S_).sum(axis=1)).ravel(), rtol=1e-13)
    assert np.allclose(D, (S_ @ S_.T).toarray(), rtol=1e-13, atol=0)
    assert 1.5 < int(oracle.flops(A, At).sum()) / P.nnz <= 4.0


# ------------------------------------------------------------------ semirings
def test_semiring_plus_times_is_the_product():
    rng = np.random.default_rng(21)
    A, B = random_sparse(30, 25, 0.2, rng), random_sparse(25, 28, 0.2, rng)
    P, Q = oracle.spgemm(A, B), oracle.spgemm_semiring(A, B, "plus_times")
    assert np.array_equal(P.colptr, Q.colptr) and np.array_equal(P.rowidx, Q.rowidx)
    assert np.allclose(P.values, Q.values, rtol=1e-13, atol=0)


def test_semiring_or_and_is_the_pattern_product():
    rng = np.random.default_rng(22)
    A, B = random_sparse(40, 30, 0.1, rng), random_sparse(30, 35, 0.1, rng)
    Q = oracle.spgemm_semiring(A, B, "or_and")
    want = (pattern_dense(A).astype(np.int64) @ pattern_dense(B).astype(np.int64)) > 0
    got = np.zeros_like(want)
    for j in range(Q.ncols):
        got[Q.rowidx[Q.colptr[j]:Q.colptr[j + 1]], j] = True
    assert np.array_equal(got, want) and np.all(Q.values == 1.0)


def test_semiring_min_plus_squaring_reaches_shortest_paths():
    """Repeated min-plus squaring of a weight matrix with a zero diagonal
    gives distances over at most 2^t edges; after ceil(log2 n) squarings they
    are the all-pairs shortest paths (scipy's Dijkstra)."""
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(23)
    n = 24
    mask = rng.random((n, n)) < 0.12
    np.fill_diagonal(mask, False)
    Wd = np.where(mask, rng.integers(1, 10, (n, n)).astype(np.float64), 0.0)
    D = Wd.copy()
    np.fill_diagonal(D, 0.0)
    # the zero diagonal must be stored: the pattern is mask | I
    pat = mask | np.eye(n, dtype=bool)
    colptr = np.concatenate([[0], np.cumsum(pat.sum(0))]).astype(np.int64)
    rows = np.concatenate([np.nonzero(pat[:, j])[0] for j in range(n)]).astype(np.int32)
    vals = np.concatenate([D[pat[:, j], j] for j in range(n)])
    M = Mat(n, n, colptr, rows, vals)
    for _ in range(int(np.ceil(np.log2(n)))):
        M = oracle.spgemm_semiring(M, M, "min_plus")
    got = np.full((n, n), np.inf)
    for j in range(n):
        got[M.rowidx[M.colptr[j]:M.colptr[j + 1]], j] = M.values[M.colptr[j]:M.colptr[j + 1]]
    # entry (i, j) of the column-oriented product is the path i <- j, i.e. from j to i along W(i, k) W(k, j)
    want = shortest_path(sp.csr_matrix(Wd.T), method="D", directed=True).T
    assert np.array_equal(got, want)


def test_semiring_min_plus_two_hops_by_hand():
    # edges 0->1 (2), 1->2 (3), 0->2 (7): stored as W(dst, src); two hops from 0 to 2 cost 5
    W = Mat(3, 3, np.array([0, 2, 3, 3]), np.array([1, 2, 2], np.int32), np.array([2.0, 7.0, 3.0]))
    Q = oracle.spgemm_semiring(W, W, "min_plus")  # exactly two edges
    assert Q.colptr.tolist() == [0, 1, 1, 1] and Q.rowidx.tolist() == [2] and Q.values.tolist() == [5.0]


from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402


@settings(max_examples=120, deadline=None)
@given(st.integers(0, 10 ** 6), st.integers(0, 12), st.integers(0, 12), st.floats(-2.5, 2.5), st.floats(0, 2))
def test_prune_monotone(seed, k1, k2, t1, dt):
    """A larger k keeps a superset (the smaller kept set is a prefix of the
    larger in rank order); a higher threshold keeps a subset; counts are
    min(k, candidates) per column."""
    M = _tie_heavy(seed % 1000, m=10, n=8, dens=0.7)
    ka, kb = min(k1, k2), max(k1, k2)
    t2 = t1 + dt

    def kept(P):
        return [set(P.rowidx[P.colptr[j]:P.colptr[j + 1]].tolist()) for j in range(P.ncols)]

    Pa, Pb = oracle.prune_topk(M, t1, ka), oracle.prune_topk(M, t1, kb)
    assert all(x <= y for x, y in zip(kept(Pa), kept(Pb)))
    Ph = oracle.prune_topk(M, t2, kb)
    Pl = oracle.prune_topk(M, t1, -1)
    Phl = oracle.prune_topk(M, t2, -1)
    assert all(x <= y for x, y in zip(kept(Phl), kept(Pl)))
    for j in range(M.ncols):
        v = M.values[M.colptr[j]:M.colptr[j + 1]]
        ncand = int((v >= t2).sum())
        assert Ph.colptr[j + 1] - Ph.colptr[j] == min(kb, ncand)
