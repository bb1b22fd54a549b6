"""ctypes binding of libspc5.so (the C ABI in include/spc5.h).

Argument marshalling only: every computation runs in the HIP library.  Torch
supplies device memory (tensors' data_ptr()) and the current HIP stream.
If the library is not built the calls raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspc5.so")

SPC5_F64, SPC5_F32 = 0, 1
KERNEL_AUTO, KERNEL_ROWS, KERNEL_SWEEP, KERNEL_STAGED = 0, 1, 2, 3
STATUS = {0: "SPC5_OK", -1: "SPC5_EINVAL", -2: "SPC5_EBADCSR", -3: "SPC5_ENOMEM",
          -4: "SPC5_EDEVICE", -5: "SPC5_EUNSUPPORTED"}

# every symbol include/spc5.h declares
EXPORTS = [
    "csr_to_spc5", "spc5_free", "spc5_get_info", "spc5_export", "spc5_to_csr",
    "spc5_set_schedule",
    "spc5_set_variant",
    "spc5_spmv", "spc5_spmv_noalloc", "spc5_spmv_values", "spc5_spmv_transpose",
    "spc5_spmv_transpose_values",
    "spc5_prepare_transpose", "spc5_values_grad", "spc5_spmm", "spc5_batch_create", "spc5_batch_free",
    "spc5_set_batch_schedule",
    "spc5_batch_set_operands", "spc5_batch_run", "spc5_batch_spmm", "spc5_plan",
    "spc5_csr_create", "spc5_csr_free", "spc5_csr_spmv",
    "spc5_csr_bytes", "spc5_last_error", "spc5_version",
]


class Spc5Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class spc5_info(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nblocks", ctypes.c_int64), ("npanels", ctypes.c_int64),
                ("r", ctypes.c_int32), ("c", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("mask_bytes", ctypes.c_int32), ("panels_per_tile", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("ntiles", ctypes.c_int64),
                ("max_panel_blocks", ctypes.c_int64),
                ("fill", ctypes.c_double), ("spmv_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("transpose_r", ctypes.c_int),
                ("transpose_c", ctypes.c_int), ("transpose_kernel", ctypes.c_int),
                ("variant", ctypes.c_int), ("transpose_bytes", ctypes.c_int64),
                ("split_panels", ctypes.c_int64)]


_lib = None


def lib():
    """Load libspc5.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2307_14774_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.csr_to_spc5.argtypes = [I64, I64, P, P, P, I, I, I, ctypes.POINTER(P)]
        L.spc5_free.argtypes = [P]
        L.spc5_free.restype = None
        L.spc5_get_info.argtypes = [P, ctypes.POINTER(spc5_info)]
        L.spc5_export.argtypes = [P, P, P, P, P]
        L.spc5_to_csr.argtypes = [P, P, P, P]
        L.spc5_set_schedule.argtypes = [P, I, I]
        L.spc5_set_variant.argtypes = [P, I]
        L.spc5_spmv.argtypes = [P, P, P, P]
        L.spc5_spmv_values.argtypes = [P, P, P, P, P]
        L.spc5_spmv_noalloc.argtypes = [P, P, P, P]
        L.spc5_spmv_transpose.argtypes = [P, P, P, P]
        L.spc5_spmv_transpose_values.argtypes = [P, P, P, P, P]
        L.spc5_values_grad.argtypes = [P, P, P, P, P]
        L.spc5_prepare_transpose.argtypes = [P, I, I]
        L.spc5_spmm.argtypes = [P, I, P, P, P]
        L.spc5_batch_create.argtypes = [I, P, ctypes.POINTER(P)]
        L.spc5_set_batch_schedule.argtypes = [P, I]
        L.spc5_batch_free.argtypes = [P]
        L.spc5_batch_free.restype = None
        L.spc5_batch_spmm.argtypes = [P, I, P, P, P]
        L.spc5_batch_set_operands.argtypes = [P, I, P, P]
        L.spc5_batch_run.argtypes = [P, P]
        L.spc5_plan.argtypes = [I64, I64, P, P, I, P, P, P]
        L.spc5_csr_create.argtypes = [I64, I64, P, P, P, I, ctypes.POINTER(P)]
        L.spc5_csr_free.argtypes = [P]
        L.spc5_csr_free.restype = None
        L.spc5_csr_spmv.argtypes = [P, P, P, P]
        L.spc5_csr_bytes.argtypes = [P]
        L.spc5_csr_bytes.restype = I64
        L.spc5_last_error.restype = ctypes.c_char_p
        L.spc5_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise Spc5Error(st, lib().spc5_last_error().decode())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(dtype) -> int:
    s = str(dtype)
    if s in ("float64", "torch.float64", "f64", "<f8"):
        return SPC5_F64
    if s in ("float32", "torch.float32", "f32", "<f4"):
        return SPC5_F32
    raise ValueError(f"unsupported dtype {dtype}")


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_code: int, numel: int, name: str):
    """Checked data_ptr of a contiguous device tensor of the given dtype/size."""
    import torch
    want = torch.float64 if dtype_code == SPC5_F64 else torch.float32
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Spc5Matrix:
    """A beta(r,c) matrix resident on the device (owns a spc5_matrix*)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self.info = self._info()

    # -- creation ---------------------------------------------------------
    @classmethod
    def from_csr(cls, rowptr, colidx, values, ncols: int, r: int, c: int,
                 dtype="float64") -> "Spc5Matrix":
        code = _dtype_code(dtype)
        npdt = np.float64 if code == SPC5_F64 else np.float32
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=npdt)
        h = ctypes.c_void_p()
        _check(lib().csr_to_spc5(rowptr.shape[0] - 1, ncols, _np_ptr(rowptr), _np_ptr(colidx),
                                 _np_ptr(values), code, r, c, ctypes.byref(h)))
        return cls(h)

    def _info(self) -> spc5_info:
        inf = spc5_info()
        _check(lib().spc5_get_info(self._h, ctypes.byref(inf)))
        return inf

    @property
    def handle(self):
        return self._h

    @property
    def dtype_code(self) -> int:
        return self.info.dtype

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.info.dtype == SPC5_F64 else torch.float32

    @property
    def shape(self):
        return (self.info.nrows, self.info.ncols)

    def free(self):
        if self._h:
            lib().spc5_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_schedule(self, kernel: str = "auto", panels_per_tile: int = 0):
        """kernel: 'auto', 'staged', 'rows' or 'sweep'; panels_per_tile: tile
        width of the staged and sweep kernels (0 = default)."""
        code = {"auto": KERNEL_AUTO, "rows": KERNEL_ROWS, "sweep": KERNEL_SWEEP,
                "staged": KERNEL_STAGED}[kernel]
        _check(lib().spc5_set_schedule(self._h, code, panels_per_tile))
        self.info = self._info()

    def set_batch_schedule(self, panels_per_tile: int = 0):
        """Tile cap (panels) this matrix gets in batches built afterwards;
        0 restores the default."""
        _check(lib().spc5_set_batch_schedule(self._h, panels_per_tile))

    def set_variant(self, partial_x: bool = False, row_reduce: bool = False,
                    union_x: bool = False):
        """Ablation variants of the staged kernel (partial x load, per-row
        reduction, x load by the merged row predicates); all False restores
        the default."""
        flags = (1 if partial_x else 0) | (2 if row_reduce else 0) | (4 if union_x else 0)
        _check(lib().spc5_set_variant(self._h, flags))
        self.info = self._info()

    @property
    def kernel(self) -> str:
        return {KERNEL_ROWS: "rows", KERNEL_SWEEP: "sweep",
                KERNEL_STAGED: "staged"}[self.info.kernel]

    def export(self):
        """Host copies of (blk_ptr int64, blk_col int32, masks uint8/16, values)."""
        inf = self.info
        bp = np.zeros(inf.npanels + 1, dtype=np.int64)
        bc = np.zeros(inf.nblocks, dtype=np.int32)
        mk = np.zeros(inf.nblocks * inf.r, dtype=np.uint8 if inf.mask_bytes == 1 else np.uint16)
        va = np.zeros(inf.nnz, dtype=np.float64 if inf.dtype == SPC5_F64 else np.float32)
        _check(lib().spc5_export(self._h, _np_ptr(bp), _np_ptr(bc), _np_ptr(mk), _np_ptr(va)))
        return bp, bc, mk, va

    def to_csr(self):
        """Host CSR (rowptr int64, colidx int32, values) read back from the
        device arrays (the inverse conversion)."""
        inf = self.info
        rp = np.zeros(inf.nrows + 1, dtype=np.int64)
        ci = np.zeros(inf.nnz, dtype=np.int32)
        va = np.zeros(inf.nnz, dtype=np.float64 if inf.dtype == SPC5_F64 else np.float32)
        _check(lib().spc5_to_csr(self._h, _np_ptr(rp), _np_ptr(ci), _np_ptr(va)))
        return rp, ci, va

    # -- compute ----------------------------------------------------------
    def spmv(self, x, y=None, stream=None):
        import torch
        inf = self.info
        if y is None:
            y = torch.empty(inf.nrows, dtype=self.torch_dtype, device=x.device)
        _check(lib().spc5_spmv(self._h, _dev_ptr(x, inf.dtype, inf.ncols, "x"),
                               _dev_ptr(y, inf.dtype, inf.nrows, "y"), _stream(stream)))
        return y

    def spmv_noalloc(self, x, y, stream=None):
        """y = A x through the allocation-free entry point (piece-tile partial
        sums in the library's fixed device array); y must be given."""
        inf = self.info
        _check(lib().spc5_spmv_noalloc(self._h, _dev_ptr(x, inf.dtype, inf.ncols, "x"),
                                       _dev_ptr(y, inf.dtype, inf.nrows, "y"), _stream(stream)))
        return y

    def spmv_values(self, values, x, y=None, stream=None):
        import torch
        inf = self.info
        if y is None:
            y = torch.empty(inf.nrows, dtype=self.torch_dtype, device=x.device)
        _check(lib().spc5_spmv_values(self._h, _dev_ptr(values, inf.dtype, inf.nnz, "values"),
                                      _dev_ptr(x, inf.dtype, inf.ncols, "x"),
                                      _dev_ptr(y, inf.dtype, inf.nrows, "y"), _stream(stream)))
        return y

    def prepare_transpose(self, r: int = 0, c: int = 0):
        """Build the transposed-product plan (A^T stored in beta(r,c), 0 = own
        shape): transposes then run as forward products, without atomics."""
        _check(lib().spc5_prepare_transpose(self._h, r, c))
        self.info = self._info()

    @property
    def has_transpose_plan(self) -> bool:
        return self.info.transpose_r > 0

    def transpose(self, ybar, xbar=None, values=None, stream=None):
        import torch
        inf = self.info
        if xbar is None:
            xbar = torch.empty(inf.ncols, dtype=self.torch_dtype, device=ybar.device)
        vp = None if values is None else _dev_ptr(values, inf.dtype, inf.nnz, "values")
        _check(lib().spc5_spmv_transpose_values(
            self._h, vp, _dev_ptr(ybar, inf.dtype, inf.nrows, "ybar"),
            _dev_ptr(xbar, inf.dtype, inf.ncols, "xbar"), _stream(stream)))
        return xbar

    def values_grad(self, ybar, x, vbar=None, stream=None):
        import torch
        inf = self.info
        if vbar is None:
            vbar = torch.empty(inf.nnz, dtype=self.torch_dtype, device=x.device)
        _check(lib().spc5_values_grad(self._h, _dev_ptr(ybar, inf.dtype, inf.nrows, "ybar"),
                                      _dev_ptr(x, inf.dtype, inf.ncols, "x"),
                                      _dev_ptr(vbar, inf.dtype, inf.nnz, "vbar"),
                                      _stream(stream)))
        return vbar

    def spmm(self, X, Y=None, stream=None):
        import torch
        inf = self.info
        if X.dim() != 2 or X.shape[0] != inf.ncols:
            raise ValueError("X must be (ncols, k)")
        k = X.shape[1]
        if Y is None:
            Y = torch.empty((inf.nrows, k), dtype=self.torch_dtype, device=X.device)
        _check(lib().spc5_spmm(self._h, k, _dev_ptr(X, inf.dtype, inf.ncols * k, "X"),
                               _dev_ptr(Y, inf.dtype, inf.nrows * k, "Y"), _stream(stream)))
        return Y


class CsrMatrix:
    """Plain CSR matrix on the device (the comparison kernel)."""

    def __init__(self, rowptr, colidx, values, ncols: int, dtype="float64"):
        code = _dtype_code(dtype)
        npdt = np.float64 if code == SPC5_F64 else np.float32
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=npdt)
        self.nrows, self.ncols, self.nnz = rowptr.shape[0] - 1, ncols, int(rowptr[-1])
        self.dtype_code = code
        h = ctypes.c_void_p()
        _check(lib().spc5_csr_create(self.nrows, ncols, _np_ptr(rowptr), _np_ptr(colidx),
                                     _np_ptr(values), code, ctypes.byref(h)))
        self._h = h
        self.spmv_bytes = int(lib().spc5_csr_bytes(self._h))

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype_code == SPC5_F64 else torch.float32

    def spmv(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.nrows, dtype=self.torch_dtype, device=x.device)
        _check(lib().spc5_csr_spmv(self._h, _dev_ptr(x, self.dtype_code, self.ncols, "x"),
                                   _dev_ptr(y, self.dtype_code, self.nrows, "y"),
                                   _stream(stream)))
        return y

    def free(self):
        if self._h:
            lib().spc5_csr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# C-ABI names, for callers that prefer them
def csr_to_spc5(rowptr, colidx, values, ncols, r, c, dtype="float64") -> Spc5Matrix:
    return Spc5Matrix.from_csr(rowptr, colidx, values, ncols, r, c, dtype)


def spc5_spmv(A: Spc5Matrix, x, y, stream=None):
    return A.spmv(x, y, stream)


def spc5_spmv_transpose(A: Spc5Matrix, ybar, xbar, stream=None):
    return A.transpose(ybar, xbar, stream=stream)


def spc5_free(A: Spc5Matrix):
    A.free()


def plan(rowptr, colidx, ncols: int, candidates):
    """Block counts of the CSR matrix for each candidate (r, c), counted on the
    device without converting (spc5_plan)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    rs = np.ascontiguousarray([r for r, _ in candidates], dtype=np.int32)
    cs = np.ascontiguousarray([c for _, c in candidates], dtype=np.int32)
    out = np.zeros(len(candidates), dtype=np.int64)
    _check(lib().spc5_plan(rowptr.shape[0] - 1, ncols, _np_ptr(rowptr), _np_ptr(colidx),
                           len(candidates), _np_ptr(rs), _np_ptr(cs), _np_ptr(out)))
    return [int(v) for v in out]


class Spc5Batch:
    """Several matrices of one dtype, multiplied in one persistent launch."""

    def __init__(self, mats):
        self.mats = list(mats)
        arr = (ctypes.c_void_p * len(self.mats))(*[m.handle for m in self.mats])
        h = ctypes.c_void_p()
        _check(lib().spc5_batch_create(len(self.mats), arr, ctypes.byref(h)))
        self._h = h
        self._bound = None

    def set_operands(self, Xs, Ys):
        """Xs[m]: (ncols_m, k) device tensors, Ys[m]: (nrows_m, k); same k."""
        if len(Xs) != len(self.mats) or len(Ys) != len(self.mats):
            raise ValueError("one X and one Y per matrix")
        k = Xs[0].shape[1]
        xp, yp = [], []
        for M, X, Y in zip(self.mats, Xs, Ys):
            inf = M.info
            if X.dim() != 2 or X.shape[1] != k or Y.dim() != 2 or Y.shape[1] != k:
                raise ValueError("X and Y must be 2-D with the same number of columns")
            xp.append(_dev_ptr(X, inf.dtype, inf.ncols * k, "X").value)
            yp.append(_dev_ptr(Y, inf.dtype, inf.nrows * k, "Y").value)
        xa = (ctypes.c_void_p * len(xp))(*xp)
        ya = (ctypes.c_void_p * len(yp))(*yp)
        _check(lib().spc5_batch_set_operands(self._h, k, xa, ya))
        self._bound = (list(Xs), list(Ys))   # keep the tensors alive

    def run(self, stream=None):
        _check(lib().spc5_batch_run(self._h, _stream(stream)))

    def spmm(self, Xs, Ys=None, stream=None):
        import torch
        if Ys is None:
            Ys = [torch.empty((M.info.nrows, X.shape[1]), dtype=M.torch_dtype, device=X.device)
                  for M, X in zip(self.mats, Xs)]
        self.set_operands(Xs, Ys)
        self.run(stream)
        return Ys

    def free(self):
        if self._h:
            lib().spc5_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
