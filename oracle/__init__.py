"""SPC5 oracle: plain FP64 CPU reference (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path never calls it and shares no code with it.

The arithmetic lives in ``spc5_oracle.c`` (built with ``-O3 -ffp-contract=off``
so every product is rounded before it is added, and with OpenMP for the
threaded host-baseline form of O1).  This module only marshals numpy
arrays to it, plus a few dense helpers used on tiny cases.

Functions and the passage of arXiv 2307.14774 each one follows:

* ``csr_spmv``          -- O1, y = A x by the CSR definition (Section 2.3).
* ``csr_spmv_par``      -- O1 with its rows split over CPU threads (host
                           baseline only; bitwise equal to ``csr_spmv``).
* ``csr_spmm``          -- O1 over several right-hand sides.
* ``csr_spmv_t``        -- O2, xbar = A^T ybar by definition.
* ``csr_to_spc5``       -- O3, greedy beta(r,c) blocking (Section 2.4).
* ``spc5_to_csr``       -- O4, inverse expansion (Fig. 2 caption).
* ``spc5_spmv``         -- O5, the beta(r,c) product by the format's
                           definition: O4 to CSR, then O1 (Section 2.4).
* ``spc5_values_grad``  -- O6, d<ybar, A(theta) x>/d theta in packed order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spc5_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction, no fast-math;
    OpenMP only spreads whole rows of the host-baseline O1 over threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.oracle_csr_spmv.argtypes = [I64, P, P, P, P, P]
        lib.oracle_csr_spmv_par.argtypes = [I64, P, P, P, P, P, I]
        lib.oracle_csr_spmm.argtypes = [I64, P, P, P, I64, P, P]
        lib.oracle_csr_spmv_t.argtypes = [I64, I64, P, P, P, P, P]
        lib.oracle_spc5_count.argtypes = [I64, P, P, I, I, P]
        lib.oracle_spc5_count.restype = I64
        lib.oracle_csr_to_spc5.argtypes = [I64, P, P, P, I, I, P, P, P, P]
        lib.oracle_spc5_to_csr.argtypes = [I64, I, I, P, P, P, P, P, P, P]
        lib.oracle_spc5_spmv.argtypes = [I64, I, I, P, P, P, P, P, P]
        lib.oracle_spc5_values_grad.argtypes = [I64, I, I, P, P, P, P, P, P]
        for f in ("oracle_csr_spmv", "oracle_csr_spmv_par", "oracle_csr_spmm", "oracle_csr_spmv_t",
                  "oracle_csr_to_spc5", "oracle_spc5_to_csr", "oracle_spc5_spmv",
                  "oracle_spc5_values_grad"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(rowptr, colidx, values):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.float64)
    return rowptr, colidx, values


@dataclass
class Spc5:
    """SPC5 beta(r,c) arrays as produced by the oracle converter."""
    nrows: int
    ncols: int
    r: int
    c: int
    blk_ptr: np.ndarray   # int64[npanels+1]
    blk_col: np.ndarray   # int32[nblocks]
    masks: np.ndarray     # uint16[nblocks*r], index b*r+i
    values: np.ndarray    # float64[nnz], packed order

    @property
    def npanels(self) -> int:
        return (self.nrows + self.r - 1) // self.r

    @property
    def nblocks(self) -> int:
        return int(self.blk_col.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.values.shape[0])


def csr_spmv(rowptr, colidx, values, x) -> np.ndarray:
    rowptr, colidx, values = _csr_arrays(rowptr, colidx, values)
    x = np.ascontiguousarray(x, dtype=np.float64)
    nrows = rowptr.shape[0] - 1
    y = np.empty(nrows, dtype=np.float64)
    _load().oracle_csr_spmv(nrows, _p(rowptr), _p(colidx), _p(values), _p(x), _p(y))
    return y


def csr_spmv_par(rowptr, colidx, values, x, nthreads: int) -> np.ndarray:
    """O1 with the rows cut into `nthreads` equal contiguous ranges, one per
    thread (host baseline only)."""
    rowptr, colidx, values = _csr_arrays(rowptr, colidx, values)
    x = np.ascontiguousarray(x, dtype=np.float64)
    nrows = rowptr.shape[0] - 1
    y = np.empty(nrows, dtype=np.float64)
    _load().oracle_csr_spmv_par(nrows, _p(rowptr), _p(colidx), _p(values), _p(x), _p(y),
                                int(nthreads))
    return y


def csr_spmm(rowptr, colidx, values, X) -> np.ndarray:
    """X: (ncols, k) row-major; returns (nrows, k)."""
    rowptr, colidx, values = _csr_arrays(rowptr, colidx, values)
    X = np.ascontiguousarray(X, dtype=np.float64)
    nrows = rowptr.shape[0] - 1
    k = X.shape[1]
    Y = np.empty((nrows, k), dtype=np.float64)
    _load().oracle_csr_spmm(nrows, _p(rowptr), _p(colidx), _p(values), k, _p(X), _p(Y))
    return Y


def csr_spmv_t(rowptr, colidx, values, ybar, ncols: int) -> np.ndarray:
    rowptr, colidx, values = _csr_arrays(rowptr, colidx, values)
    ybar = np.ascontiguousarray(ybar, dtype=np.float64)
    nrows = rowptr.shape[0] - 1
    xbar = np.empty(ncols, dtype=np.float64)
    _load().oracle_csr_spmv_t(nrows, ncols, _p(rowptr), _p(colidx), _p(values),
                              _p(ybar), _p(xbar))
    return xbar


def spc5_count(rowptr, colidx, r: int, c: int, per_panel: bool = False):
    rowptr, colidx, _ = _csr_arrays(rowptr, colidx, np.zeros(0))
    nrows = rowptr.shape[0] - 1
    npanels = (nrows + r - 1) // r
    cnt = np.empty(max(npanels, 1), dtype=np.int64)
    total = _load().oracle_spc5_count(nrows, _p(rowptr), _p(colidx), r, c, _p(cnt))
    return (int(total), cnt[:npanels]) if per_panel else int(total)


def csr_to_spc5(rowptr, colidx, values, ncols: int, r: int, c: int) -> Spc5:
    if not (1 <= r <= 8 and 1 <= c <= 16):
        raise ValueError("oracle supports 1 <= r <= 8, 1 <= c <= 16")
    rowptr, colidx, values = _csr_arrays(rowptr, colidx, values)
    nrows = rowptr.shape[0] - 1
    nnz = int(rowptr[-1])
    nblocks = spc5_count(rowptr, colidx, r, c)
    npanels = (nrows + r - 1) // r
    blk_ptr = np.zeros(npanels + 1, dtype=np.int64)
    blk_col = np.zeros(nblocks, dtype=np.int32)
    masks = np.zeros(nblocks * r, dtype=np.uint16)
    packed = np.zeros(nnz, dtype=np.float64)
    _load().oracle_csr_to_spc5(nrows, _p(rowptr), _p(colidx), _p(values), r, c,
                               _p(blk_ptr), _p(blk_col), _p(masks), _p(packed))
    return Spc5(nrows, ncols, r, c, blk_ptr, blk_col, masks, packed)


def spc5_to_csr(S: Spc5):
    nnz = S.nnz
    rowptr = np.zeros(S.nrows + 1, dtype=np.int64)
    colidx = np.zeros(nnz, dtype=np.int32)
    values = np.zeros(nnz, dtype=np.float64)
    blk_ptr = np.ascontiguousarray(S.blk_ptr, dtype=np.int64)
    blk_col = np.ascontiguousarray(S.blk_col, dtype=np.int32)
    masks = np.ascontiguousarray(S.masks, dtype=np.uint16)
    packed = np.ascontiguousarray(S.values, dtype=np.float64)
    _load().oracle_spc5_to_csr(S.nrows, S.r, S.c, _p(blk_ptr), _p(blk_col), _p(masks),
                               _p(packed), _p(rowptr), _p(colidx), _p(values))
    return rowptr, colidx, values


def spc5_spmv(S: Spc5, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(S.nrows, dtype=np.float64)
    blk_ptr = np.ascontiguousarray(S.blk_ptr, dtype=np.int64)
    blk_col = np.ascontiguousarray(S.blk_col, dtype=np.int32)
    masks = np.ascontiguousarray(S.masks, dtype=np.uint16)
    packed = np.ascontiguousarray(S.values, dtype=np.float64)
    _load().oracle_spc5_spmv(S.nrows, S.r, S.c, _p(blk_ptr), _p(blk_col), _p(masks),
                             _p(packed), _p(x), _p(y))
    return y


def spc5_values_grad(S: Spc5, ybar, x) -> np.ndarray:
    ybar = np.ascontiguousarray(ybar, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    vbar = np.empty(S.nnz, dtype=np.float64)
    blk_ptr = np.ascontiguousarray(S.blk_ptr, dtype=np.int64)
    blk_col = np.ascontiguousarray(S.blk_col, dtype=np.int32)
    masks = np.ascontiguousarray(S.masks, dtype=np.uint16)
    _load().oracle_spc5_values_grad(S.nrows, S.r, S.c, _p(blk_ptr), _p(blk_col),
                                    _p(masks), _p(ybar), _p(x), _p(vbar))
    return vbar


def dense(rowptr, colidx, values, ncols: int) -> np.ndarray:
    """Dense copy of a CSR matrix (tiny cases only)."""
    nrows = len(rowptr) - 1
    A = np.zeros((nrows, ncols), dtype=np.float64)
    for i in range(nrows):
        for k in range(int(rowptr[i]), int(rowptr[i + 1])):
            A[i, int(colidx[k])] = values[k]
    return A


def rel_l2(y, yref) -> float:
    """Relative L2 error ||y - yref|| / ||yref|| (0 when both are zero)."""
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    den = float(np.linalg.norm(yref))
    num = float(np.linalg.norm(y - yref))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den
