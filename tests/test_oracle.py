"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: each check uses an independent
route (dense numpy/scipy products, exact rational or integer arithmetic, brute
force on tiny inputs, closed forms of the stencil block counts, the paper's own
worked captions and table entries).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2307_14774_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SHAPES = [(1, 8), (2, 4), (4, 4), (1, 16), (2, 8), (4, 8), (8, 8), (3, 5), (1, 1),
          (8, 16), (5, 3), (7, 16), (2, 1)]


def tiny_cases():
    out = []
    seed = 0
    for (m, n) in [(1, 1), (3, 7), (7, 3), (16, 16), (33, 20), (20, 65), (64, 64)]:
        for dens in (0.0, 0.05, 0.3, 0.8, 1.0):
            out.append(W.random_sparse(m, n, dens, seed=seed))
            seed += 1
    return out


# ---------------------------------------------------------------- O1: CSR SpMV

@pytest.mark.parametrize("A", tiny_cases(), ids=lambda a: a.name)
def test_csr_spmv_vs_dense_and_scipy(A):
    y = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    D = np.zeros((A.nrows, A.ncols))
    rows = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
    D[rows, A.colidx] = A.values
    np.testing.assert_allclose(y, D @ A.x, rtol=1e-13, atol=1e-13)
    S = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(A.nrows, A.ncols))
    np.testing.assert_allclose(y, S @ A.x, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_csr_spmv_integer_exact(seed):
    # Small integers keep every partial sum exact, so the result is unique.
    A = W.random_sparse(40, 57, 0.3, seed=seed, integer=True)
    y = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    for i in range(A.nrows):
        exact = 0
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            exact += int(A.values[k]) * int(A.x[A.colidx[k]])
        assert y[i] == exact


def test_csr_spmv_unit_vectors_give_columns():
    A = W.random_sparse(30, 25, 0.4, seed=3)
    D = np.zeros((A.nrows, A.ncols))
    rows = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
    D[rows, A.colidx] = A.values
    for j in range(A.ncols):
        e = np.zeros(A.ncols)
        e[j] = 1.0
        y = oracle.csr_spmv(A.rowptr, A.colidx, A.values, e)
        assert np.array_equal(y, D[:, j])


def test_csr_spmv_linearity():
    A = W.random_sparse(50, 60, 0.2, seed=4)
    rng = np.random.default_rng(1)
    x1, x2 = rng.uniform(-1, 1, 60), rng.uniform(-1, 1, 60)
    a, b = 0.75, -1.5
    lhs = oracle.csr_spmv(A.rowptr, A.colidx, A.values, a * x1 + b * x2)
    rhs = a * oracle.csr_spmv(A.rowptr, A.colidx, A.values, x1) + \
        b * oracle.csr_spmv(A.rowptr, A.colidx, A.values, x2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


def test_csr_spmv_higham_bound():
    """|y_hat_i - y_i| <= gamma_n * sum_j |a_ij x_j|, exact y_i by rationals."""
    u = 2.0 ** -53
    A = W.random_sparse(25, 40, 0.5, seed=7)
    y = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    for i in range(A.nrows):
        lo, hi = A.rowptr[i], A.rowptr[i + 1]
        exact = sum((Fraction(float(A.values[k])) * Fraction(float(A.x[A.colidx[k]]))
                     for k in range(lo, hi)), Fraction(0))
        n = hi - lo
        gamma = n * u / (1 - n * u)
        absum = sum(abs(float(A.values[k]) * float(A.x[A.colidx[k]])) for k in range(lo, hi))
        assert abs(Fraction(float(y[i])) - exact) <= Fraction(gamma * absum * (1 + 1e-12))


def test_csr_spmm_columns():
    A = W.random_sparse(31, 29, 0.3, seed=11)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (29, 5))
    Y = oracle.csr_spmm(A.rowptr, A.colidx, A.values, X)
    S = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(31, 29))
    np.testing.assert_allclose(Y, S @ X, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- O2: transpose

@pytest.mark.parametrize("A", tiny_cases()[::3], ids=lambda a: a.name)
def test_transpose_vs_dense(A):
    rng = np.random.default_rng(5)
    w = rng.uniform(-1, 1, A.nrows)
    xb = oracle.csr_spmv_t(A.rowptr, A.colidx, A.values, w, A.ncols)
    S = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(A.nrows, A.ncols))
    np.testing.assert_allclose(xb, S.T @ w, rtol=1e-13, atol=1e-13)


def test_transpose_adjoint_and_unit_rows():
    A = W.random_sparse(40, 33, 0.25, seed=9)
    rng = np.random.default_rng(6)
    w = rng.uniform(-1, 1, 40)
    xb = oracle.csr_spmv_t(A.rowptr, A.colidx, A.values, w, 33)
    y = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    assert abs(np.dot(w, y) - np.dot(xb, A.x)) <= 1e-12 * (np.abs(w) @ np.abs(y) + 1)
    for i in range(A.nrows):
        e = np.zeros(40)
        e[i] = 1.0
        row = oracle.csr_spmv_t(A.rowptr, A.colidx, A.values, e, 33)
        ref = np.zeros(33)
        ref[A.colidx[A.rowptr[i]:A.rowptr[i + 1]]] = A.values[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.array_equal(row, ref)


# ---------------------------------------------------------------- O3/O4: format

def edge_cases():
    cases = []
    z = np.zeros
    # empty matrices
    cases.append(W.Csr(0, 0, z(1, np.int64), z(0, np.int32), z(0), z(0), "empty0x0"))
    cases.append(W.Csr(5, 0, z(6, np.int64), z(0, np.int32), z(0), z(0), "5x0"))
    cases.append(W.Csr(0, 7, z(1, np.int64), z(0, np.int32), z(0), z(7), "0x7"))
    cases.append(W.Csr(9, 9, z(10, np.int64), z(0, np.int32), z(0), np.ones(9), "nnz0"))
    # one nonzero in the last column, rows not a multiple of r
    cases.append(W.Csr(7, 13, np.array([0, 0, 0, 0, 0, 0, 0, 1]), np.array([12], np.int32),
                       np.array([2.5]), np.arange(13.0), "lastcol"))
    # ncols < c, full dense rows, explicit zeros
    d = W.dense(3, seed=1)
    d.values[4] = 0.0
    d.name = "dense3_expzero"
    cases.append(d)
    cases.append(W.dense(17, seed=2))
    # all-empty panels in the middle
    rp = np.array([0, 3, 3, 3, 3, 3, 3, 3, 3, 6], dtype=np.int64)
    cases.append(W.Csr(9, 40, rp, np.array([0, 1, 39, 5, 20, 38], np.int32),
                       np.arange(1.0, 7.0), np.linspace(-1, 1, 40), "holes"))
    cases.extend(tiny_cases()[::2])
    return cases


def popcount16(m):
    return sum(bin(int(v)).count("1") for v in m)


@pytest.mark.parametrize("A", edge_cases(), ids=lambda a: a.name)
@pytest.mark.parametrize("rc", SHAPES, ids=lambda t: "b%d_%d" % t)
def test_round_trip_and_invariants(A, rc):
    r, c = rc
    S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
    # inverse gives the input back, bit for bit
    rp, ci, va = oracle.spc5_to_csr(S)
    assert np.array_equal(rp, A.rowptr)
    assert np.array_equal(ci, A.colidx)
    assert np.array_equal(va.view(np.uint64), A.values.view(np.uint64))
    # one bit per nonzero
    assert popcount16(S.masks) == A.nnz
    assert S.blk_ptr[0] == 0 and S.blk_ptr[-1] == S.nblocks
    assert np.all(np.diff(S.blk_ptr) >= 0)
    # masks hold c bits only; no bit points at or past ncols
    assert np.all(S.masks < (1 << c))
    for b in range(S.nblocks):
        rows_m = S.masks[b * r:(b + 1) * r].astype(np.int64)
        union = int(np.bitwise_or.reduce(rows_m)) if r else 0
        # a block starts at a nonzero: bit 0 is set in some row of the block
        assert union & 1
        # between 1 and r*c values per block
        assert 1 <= popcount16(rows_m) <= r * c
        top = max(k for k in range(c) if (union >> k) & 1)
        assert S.blk_col[b] + top < A.ncols
    # windows of one panel are disjoint and increasing
    for p in range(S.npanels):
        cols = S.blk_col[S.blk_ptr[p]:S.blk_ptr[p + 1]].astype(np.int64)
        assert np.all(np.diff(cols) >= c)
        for i in range(r):
            if p * r + i >= A.nrows:
                assert np.all(S.masks[S.blk_ptr[p] * r + i:S.blk_ptr[p + 1] * r:r] == 0)
    # beta(1,c) keeps the CSR value order (Conclusion)
    if r == 1:
        assert np.array_equal(S.values, A.values)


def min_cover(points, c):
    """Minimum number of length-c windows covering sorted integer points, by
    memoised search over every window start that covers the first point."""
    from functools import lru_cache
    pts = tuple(points)

    @lru_cache(maxsize=None)
    def f(i):
        if i == len(pts):
            return 0
        best = None
        for s in range(pts[i] - c + 1, pts[i] + 1):
            j = i
            while j < len(pts) and pts[j] < s + c:
                j += 1
            v = 1 + f(j)
            best = v if best is None else min(best, v)
        return best
    return f(0)


@pytest.mark.parametrize("rc", [(1, 4), (2, 3), (4, 4), (3, 8), (8, 5)], ids=str)
@pytest.mark.parametrize("seed", range(4))
def test_block_count_is_minimum_cover(rc, seed):
    r, c = rc
    A = W.random_sparse(24, 48, 0.15, seed=100 + seed)
    total, per = oracle.spc5_count(A.rowptr, A.colidx, r, c, per_panel=True)
    for p in range(per.shape[0]):
        cols = sorted(set(int(v) for i in range(p * r, min(p * r + r, A.nrows))
                          for v in A.colidx[A.rowptr[i]:A.rowptr[i + 1]]))
        assert per[p] == min_cover(cols, c)
    S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
    # every anchor is a column holding a nonzero of its panel
    for p in range(S.npanels):
        cols = set(int(v) for i in range(p * r, min(p * r + r, A.nrows))
                   for v in A.colidx[A.rowptr[i]:A.rowptr[i + 1]])
        for b in range(S.blk_ptr[p], S.blk_ptr[p + 1]):
            assert int(S.blk_col[b]) in cols


@pytest.mark.parametrize("N", [8, 16, 32, 48])
def test_laplacian_closed_forms(N):
    """Per grid row: an interior row of beta(1,8) needs 3 windows (north,
    centre, south), a top or bottom row 2.  With r | N a beta(2,4) panel takes
    one window per neighbour band, and a beta(4,4) panel two for the centre
    band (6 consecutive columns) plus one each for north and south."""
    A = W.laplacian_2d(N, seed=1)
    assert A.nnz == 5 * N * N - 4 * N
    assert oracle.spc5_count(A.rowptr, A.colidx, 1, 8) == 3 * N * N - 2 * N
    assert oracle.spc5_count(A.rowptr, A.colidx, 2, 4) == 3 * N * N // 2 - N
    assert oracle.spc5_count(A.rowptr, A.colidx, 4, 4) == N * N - N // 2


@pytest.mark.parametrize("n", [6, 8, 11])
def test_fem_closed_forms(n):
    """Each row couples to the x-runs of up to 9 (dz,dy) node lines; a run is
    9 consecutive columns inside the line and 6 at its ends.  Summed over the
    grid: nnz = 9 (3n-2)^3; beta(1,8) needs 2 windows for a 9-run and 1 for a
    6-run, so 3 (3n-2)^2 (2n-2); beta(1,16) needs 1 per run, 3 (3n-2)^2 n.
    Runs of neighbouring lines start 3n columns apart, so for n >= 6 no
    window reaches the next run."""
    A = W.fem_3d(n, seed=1)
    assert A.nrows == 3 * n ** 3
    assert A.nnz == 9 * (3 * n - 2) ** 3
    assert oracle.spc5_count(A.rowptr, A.colidx, 1, 8) == 3 * (3 * n - 2) ** 2 * (2 * n - 2)
    assert oracle.spc5_count(A.rowptr, A.colidx, 1, 16) == 3 * (3 * n - 2) ** 2 * n
    # diagonal dominance as generated
    S = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(A.nrows, A.ncols))
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    np.testing.assert_allclose(d, off + 1.0, rtol=1e-12)


@pytest.mark.parametrize("n", [6, 8, 10, 16])
def test_fem_closed_forms_multirow(n):
    """beta(r,c) block counts of the FEM matrix against the panel-cover closed
    form (tests/helpers.py), every shape whose r divides 3n; at n = 96 the
    form gives 46,623,720 (beta(1,8)), 35,172,280 (beta(2,4)) and 17,667,936
    (beta(4,4))."""
    from helpers import fem_block_count
    A = W.fem_3d(n, seed=1)
    for r, c in [(1, 8), (2, 4), (4, 4), (1, 16), (2, 8), (4, 8), (8, 8), (3, 5), (6, 16)]:
        if (3 * n) % r:
            continue
        assert oracle.spc5_count(A.rowptr, A.colidx, r, c) == fem_block_count(n, r, c), (r, c)
    assert fem_block_count(96, 1, 8) == 46_623_720
    assert fem_block_count(96, 2, 4) == 35_172_280
    assert fem_block_count(96, 4, 4) == 17_667_936


def test_fig3_expand_golden():
    g = json.load(open(os.path.join(GOLDEN, "fig3_expand.json")))
    S = oracle.csr_to_spc5(np.array(g["rowptr"]), np.array(g["colidx"], np.int32),
                           np.array(g["values"]), g["ncols"], g["r"], g["c"])
    e = g["expected"]
    assert S.blk_ptr.tolist() == e["blk_ptr"]
    assert S.blk_col.tolist() == e["blk_col"]
    assert S.masks.tolist() == e["masks"]
    assert S.values.tolist() == e["packed"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_table1_dense_fill(prec):
    g = json.load(open(os.path.join(GOLDEN, "table1_dense_fill.json")))
    n = 64      # same structure as the paper's 2048 (r and VS divide n)
    A = W.dense(n, seed=3)
    c = g["vs"][prec]
    for r_s, pct in g["fill_percent"][prec].items():
        r = int(r_s)
        nb = oracle.spc5_count(A.rowptr, A.colidx, r, c)
        assert nb == n * n // (r * c)
        assert round(100 * A.nnz / (nb * r * c)) == pct


@pytest.mark.parametrize("A", edge_cases() + [W.laplacian_2d(33, seed=4),
                                               W.random_sparse(1001, 700, 0.02, seed=5)],
                         ids=lambda a: a.name)
@pytest.mark.parametrize("nthreads", [1, 2, 3, 8])
def test_csr_spmv_par_bitwise(A, nthreads):
    """The threaded host-baseline O1 gives every row to one thread, which sums
    it in storage order: bitwise equal to the sequential O1, and equal to
    scipy's product within rounding."""
    y1 = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    yp = oracle.csr_spmv_par(A.rowptr, A.colidx, A.values, A.x, nthreads)
    assert np.array_equal(yp.view(np.uint64), y1.view(np.uint64))
    if A.nrows and A.ncols:
        S = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(A.nrows, A.ncols))
        np.testing.assert_allclose(yp, S @ A.x, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- O5: the beta(r,c) product

@pytest.mark.parametrize("A", edge_cases(), ids=lambda a: a.name)
@pytest.mark.parametrize("rc", SHAPES[:8], ids=lambda t: "b%d_%d" % t)
def test_spc5_product_equals_csr_definition_bitwise(A, rc):
    r, c = rc
    S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
    y5 = oracle.spc5_spmv(S, A.x)
    y1 = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    assert np.array_equal(y5.view(np.uint64), y1.view(np.uint64))


def test_spc5_product_laplacian_vs_scipy():
    A = W.laplacian_2d(40, seed=2)
    Sm = sp.csr_matrix((A.values, A.colidx, A.rowptr), shape=(A.nrows, A.ncols))
    for r, c in [(1, 8), (2, 4), (4, 4)]:
        S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
        np.testing.assert_allclose(oracle.spc5_spmv(S, A.x), Sm @ A.x, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------- O6: values grad

@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 4), (3, 5)], ids=str)
def test_values_grad_by_exact_central_difference(rc):
    """L(theta) = <w, A(theta) x> is linear in theta, so with integer data the
    central difference with h = 1 is exact."""
    r, c = rc
    A = W.random_sparse(13, 21, 0.3, seed=21, integer=True)
    S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
    rng = np.random.default_rng(3)
    w = rng.integers(-5, 6, A.nrows).astype(np.float64)
    g = oracle.spc5_values_grad(S, w, A.x)
    for k in range(S.nnz):
        Sp = oracle.Spc5(**{**S.__dict__, "values": S.values.copy()})
        Sm = oracle.Spc5(**{**S.__dict__, "values": S.values.copy()})
        Sp.values[k] += 1.0
        Sm.values[k] -= 1.0
        fd = (w @ oracle.spc5_spmv(Sp, A.x) - w @ oracle.spc5_spmv(Sm, A.x)) / 2.0
        assert g[k] == fd
