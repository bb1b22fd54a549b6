"""Seeded synthetic inputs (CSR matrices and vectors).

This module only draws inputs; it holds none of the SpMV or SPC5 arithmetic.
Tests, the benchmark and the smoke check feed the same arrays to the HIP
library and to the CPU oracle.

The paper (arXiv 2307.14774, Section 4.2 and Table 1) measures on matrices of
the SuiteSparse collection that are not available here; these generators
stand in for their shapes: a 2D Laplacian (about 5 nonzeros per row, low block
fill), a 3-dof 27-point FEM-like matrix (81 per row, high fill), a uniform
random matrix (near the worst case of one value per block), a Zipf-skewed
graph matrix and a batch of uneven matrices with power-law row lengths.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Csr:
    nrows: int
    ncols: int
    rowptr: np.ndarray          # int64[nrows+1]
    colidx: np.ndarray          # int32[nnz], strictly increasing per row
    values: np.ndarray          # float64[nnz]
    x: np.ndarray = field(default=None)   # float64[ncols], the input vector
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _finish(nrows, ncols, counts, colidx, values, x, name) -> Csr:
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Csr(nrows, ncols, rowptr, np.ascontiguousarray(colidx, dtype=np.int32),
               np.ascontiguousarray(values, dtype=np.float64),
               None if x is None else np.ascontiguousarray(x, dtype=np.float64), name)


def random_uniform(n: int = 10_000, per_row: int = 10, seed: int = 0) -> Csr:
    """n x n, `per_row` distinct uniform columns per row, values and x U(-1,1).

    Draw order: the columns row by row, then the values in CSR order, then x.
    """
    rng = np.random.default_rng(seed)
    k = min(per_row, n)
    cols = np.empty((n, k), dtype=np.int32)
    for i in range(n):
        cols[i] = np.sort(rng.choice(n, k, replace=False))
    values = rng.uniform(-1.0, 1.0, n * k)
    x = rng.uniform(-1.0, 1.0, n)
    return _finish(n, n, np.full(n, k, dtype=np.int64), cols.reshape(-1), values, x,
                   f"random{n}x{k}")


def laplacian_2d(N: int = 2048, seed: int = 0) -> Csr:
    """5-point Laplacian on an N x N grid, row i = gy*N + gx, truncated at edges.

    Diagonal 4 + U(-1e-3, 1e-3), off-diagonal -1 + U(-1e-3, 1e-3), jitter drawn
    per entry in CSR order; then x U(-1,1).
    """
    rng = np.random.default_rng(seed)
    n = N * N
    i = np.arange(n, dtype=np.int64)
    gy, gx = np.divmod(i, N)
    cand = np.stack([i - N, i - 1, i, i + 1, i + N], axis=1)
    valid = np.stack([gy > 0, gx > 0, np.ones(n, bool), gx < N - 1, gy < N - 1], axis=1)
    counts = valid.sum(axis=1)
    colidx = cand[valid].astype(np.int32)
    isdiag = np.broadcast_to(np.array([False, False, True, False, False]), (n, 5))[valid]
    jitter = rng.uniform(-1e-3, 1e-3, colidx.shape[0])
    values = np.where(isdiag, 4.0, -1.0) + jitter
    x = rng.uniform(-1.0, 1.0, n)
    return _finish(n, n, counts, colidx, values, x, f"laplacian2d_{N}")


def fem_3d(n: int = 96, dof: int = 3, seed: int = 0) -> Csr:
    """Vector-FEM-like matrix: n^3 nodes x `dof`, 27-point node stencil, so each
    node pair couples through a dense dof x dof block.

    Node m = (z*n + y)*n + x, row = dof*m + d.  Off-diagonal values i.i.d.
    N(0,1) drawn in CSR order; the diagonal is replaced by the sum of the
    absolute off-diagonal values of its row plus 1; then x U(-1,1).
    """
    rng = np.random.default_rng(seed)
    nn = n * n * n
    m = np.arange(nn, dtype=np.int64)
    z, rem = np.divmod(m, n * n)
    y, xx = np.divmod(rem, n)
    offs, valid_cols = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                offs.append(dz * n * n + dy * n + dx)
                valid_cols.append((z + dz >= 0) & (z + dz < n) & (y + dy >= 0) &
                                  (y + dy < n) & (xx + dx >= 0) & (xx + dx < n))
    valid = np.stack(valid_cols, axis=1)                     # (nn, 27)
    del valid_cols, z, y, xx, rem
    nbr = (m[:, None] + np.asarray(offs, dtype=np.int64)[None, :]).astype(np.int32)
    node_cols = (dof * nbr[:, :, None] + np.arange(dof, dtype=np.int32)[None, None, :])
    node_cols = node_cols.reshape(nn, 27 * dof)              # (nn, 27*dof)
    valid_c = np.repeat(valid, dof, axis=1)                  # (nn, 27*dof)
    del nbr
    nb = valid.sum(axis=1)                                   # neighbours per node
    counts = np.repeat(nb * dof, dof)                        # per row
    sel = np.broadcast_to(valid_c[:, None, :], (nn, dof, 27 * dof))
    colidx = np.broadcast_to(node_cols[:, None, :], (nn, dof, 27 * dof))[sel]
    del sel, node_cols, valid_c, valid
    nrows = nn * dof
    values = rng.standard_normal(colidx.shape[0])
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rows = np.repeat(np.arange(nrows, dtype=np.int32), counts)
    isdiag = colidx == rows
    del rows
    absval = np.abs(values)
    absval[isdiag] = 0.0
    offsum = np.add.reduceat(absval, rowptr[:-1]) if nrows else np.zeros(0)
    del absval
    values[isdiag] = offsum + 1.0
    del isdiag
    x = rng.uniform(-1.0, 1.0, nrows)
    return Csr(nrows, nrows, rowptr, np.ascontiguousarray(colidx, dtype=np.int32),
               values, x, f"fem3d_{n}x{dof}")


def zipf_graph(n: int = 1 << 20, mean_len: float = 16.0, s: float = 1.2,
               seed: int = 0) -> Csr:
    """Graph-like square matrix: row length Poisson(mean_len), distinct columns
    drawn with P(col = j) proportional to (j+1)^-s (identity rank -> column
    map, so the popular columns are the first ones).  Values U(-1,1) in CSR
    order, then x N(0,1).
    """
    rng = np.random.default_rng(seed)
    lengths = np.minimum(rng.poisson(mean_len, n), n).astype(np.int64)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rows_need = lengths.copy()
    keys = np.zeros(0, dtype=np.int64)
    for _ in range(200):
        if rows_need.sum() == 0:
            break
        draw_rows = np.repeat(np.arange(n, dtype=np.int64), rows_need)
        u = rng.random(draw_rows.shape[0])
        cols = np.minimum(np.searchsorted(cdf, u, side="right"), n - 1).astype(np.int64)
        keys = np.unique(np.concatenate([keys, draw_rows * n + cols]))
        have = np.bincount(keys // n, minlength=n)
        rows_need = np.maximum(lengths - have, 0)
    r_of = keys // n
    c_of = keys % n
    # a row that drew more distinct columns than its length keeps its first ones
    rank = np.arange(keys.shape[0]) - np.searchsorted(r_of, r_of, side="left")
    keep = rank < lengths[r_of]
    r_of, c_of = r_of[keep], c_of[keep]
    counts = np.bincount(r_of, minlength=n)
    values = rng.uniform(-1.0, 1.0, c_of.shape[0])
    x = rng.standard_normal(n)
    return _finish(n, n, counts, c_of.astype(np.int32), values, x, f"zipfgraph_{n}")


def dense(n: int = 2048, seed: int = 0) -> Csr:
    """Fully dense n x n stored as CSR, values and x U(-1,1)."""
    rng = np.random.default_rng(seed)
    colidx = np.tile(np.arange(n, dtype=np.int32), n)
    values = rng.uniform(-1.0, 1.0, n * n)
    x = rng.uniform(-1.0, 1.0, n)
    return _finish(n, n, np.full(n, n, dtype=np.int64), colidx, values, x, f"dense{n}")


def random_sparse(nrows: int, ncols: int, density: float, seed: int = 0,
                  integer: bool = False, lo: int = -8, hi: int = 8) -> Csr:
    """Bernoulli(density) pattern; values U(-1,1) or integers in [lo, hi]
    (x likewise).  Used for small parity and edge cases."""
    rng = np.random.default_rng(seed)
    pat = rng.random((nrows, ncols)) < density
    counts = pat.sum(axis=1)
    rr, cc = np.nonzero(pat)
    if integer:
        values = rng.integers(lo, hi + 1, rr.shape[0]).astype(np.float64)
        x = rng.integers(lo, hi + 1, ncols).astype(np.float64)
    else:
        values = rng.uniform(-1.0, 1.0, rr.shape[0])
        x = rng.uniform(-1.0, 1.0, ncols)
    return _finish(nrows, ncols, counts, cc.astype(np.int32), values, x,
                   f"rand{nrows}x{ncols}d{density}")


def runs_matrix(n: int, rng, zipf_s: float = 1.5, cap: int = 512,
                run_frac: float = 0.3) -> Csr:
    """Square n x n matrix with power-law row lengths L = min(Zipf(zipf_s), cap)
    (the literal cap: lengths above it are set to it).  About `run_frac` of a
    row's nonzeros come in runs of 2..16 consecutive columns at uniform
    starts, the rest are uniform singletons; duplicates are merged and rows
    topped up with singletons, so a row may end a few entries above L when a
    run overshoots.  Values U(-1,1); x U(-1,1).

    Draw order: L, run lengths, run starts, singleton columns, top-ups,
    values, x."""
    L = np.minimum(rng.zipf(zipf_s, n), min(cap, n)).astype(np.int64)
    want_runs = np.round(run_frac * L).astype(np.int64)
    want_runs[want_runs < 2] = 0
    nruns = (want_runs + 8) // 9                      # mean run length 9
    rrow = np.repeat(np.arange(n, dtype=np.int64), nruns)
    rlen = rng.integers(2, 17, rrow.shape[0])
    rlen = np.minimum(rlen, n)
    rstart = (rng.random(rrow.shape[0]) * (n - rlen + 1)).astype(np.int64)
    # expand runs into (row, col)
    tot = int(rlen.sum())
    rid = np.repeat(np.arange(rrow.shape[0]), rlen)
    within = np.arange(tot) - np.repeat(np.cumsum(rlen) - rlen, rlen)
    keys = rrow[rid] * n + rstart[rid] + within
    run_cnt = np.bincount(rrow, weights=rlen, minlength=n).astype(np.int64)
    nsing = np.maximum(L - run_cnt, 0)
    srow = np.repeat(np.arange(n, dtype=np.int64), nsing)
    keys = np.concatenate([keys, srow * n + rng.integers(0, n, srow.shape[0])])
    keys = np.unique(keys)
    for _ in range(20):
        have = np.bincount(keys // n, minlength=n)
        need = np.maximum(L - have, 0)
        if need.sum() == 0:
            break
        trow = np.repeat(np.arange(n, dtype=np.int64), need)
        keys = np.unique(np.concatenate([keys, trow * n + rng.integers(0, n, trow.shape[0])]))
    rows = keys // n
    counts = np.bincount(rows, minlength=n)
    values = rng.uniform(-1.0, 1.0, keys.shape[0])
    x = rng.uniform(-1.0, 1.0, n)
    return _finish(n, n, counts, (keys % n).astype(np.int32), values, x, f"runs{n}")


def batch_of_runs(nmat: int = 256, seed: int = 0, rows_lo: int = 1000,
                  rows_hi: int = 200_000) -> list:
    """`nmat` uneven matrices: n = floor(exp(U(ln rows_lo, ln rows_hi))) rows
    each (log-uniform sizes), built by runs_matrix with one child seed each
    (numpy SeedSequence(seed).spawn(nmat))."""
    children = np.random.SeedSequence(seed).spawn(nmat)
    out = []
    for m in range(nmat):
        rng = np.random.default_rng(children[m])
        n = int(np.floor(np.exp(rng.uniform(np.log(rows_lo), np.log(rows_hi)))))
        A = runs_matrix(n, rng)
        A.name = f"batch{m}_n{n}"
        out.append(A)
    return out
