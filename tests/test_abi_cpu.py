"""C-ABI checks that need no GPU: the library loads, exports every function
include/spc5.h declares, and rejects malformed input before touching the
device (the argument checks are synchronous and run first)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_14774_amd import spc5

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spc5.h")

needs_lib = pytest.mark.skipif(not os.path.exists(spc5.LIB_PATH),
                               reason="libspc5.so not built")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_lists_binding_exports():
    assert header_functions() == sorted(spc5.EXPORTS)


@needs_lib
def test_library_exports_every_symbol():
    L = ctypes.CDLL(spc5.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert b"gfx950" in spc5.lib().spc5_version()


def _create(rowptr, colidx, values, nrows, ncols, r=1, c=8, dtype=0, out=True):
    L = spc5.lib()
    h = ctypes.c_void_p(12345)
    rp = None if rowptr is None else np.ascontiguousarray(rowptr, np.int64)
    ci = None if colidx is None else np.ascontiguousarray(colidx, np.int32)
    va = None if values is None else np.ascontiguousarray(values, np.float64)
    st = L.csr_to_spc5(nrows, ncols, spc5._np_ptr(rp), spc5._np_ptr(ci), spc5._np_ptr(va),
                       dtype, r, c, ctypes.byref(h) if out else None)
    return st, h


@needs_lib
@pytest.mark.parametrize("case,status", [
    (dict(rowptr=[1, 2], colidx=[0], values=[1.0], nrows=1, ncols=3), -2),
    (dict(rowptr=[0, 2, 1], colidx=[0, 1], values=[1.0, 2.0], nrows=2, ncols=3), -2),
    (dict(rowptr=[0, 2], colidx=[1, 1], values=[1.0, 2.0], nrows=1, ncols=3), -2),
    (dict(rowptr=[0, 2], colidx=[2, 1], values=[1.0, 2.0], nrows=1, ncols=3), -2),
    (dict(rowptr=[0, 1], colidx=[3], values=[1.0], nrows=1, ncols=3), -2),
    (dict(rowptr=[0, 1], colidx=[-1], values=[1.0], nrows=1, ncols=3), -2),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=1, ncols=3, r=9), -5),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=1, ncols=3, c=17), -5),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=1, ncols=3, r=0), -5),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=1, ncols=3, dtype=7), -1),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=-1, ncols=3), -1),
    (dict(rowptr=None, colidx=[0], values=[1.0], nrows=1, ncols=3), -1),
    (dict(rowptr=[0, 1], colidx=None, values=[1.0], nrows=1, ncols=3), -1),
    (dict(rowptr=[0, 1], colidx=[0], values=None, nrows=1, ncols=3), -1),
    (dict(rowptr=[0, 1], colidx=[0], values=[1.0], nrows=1, ncols=1 << 31), -5),
    (dict(rowptr=[0, 1 << 31], colidx=[0], values=[1.0], nrows=1, ncols=3), -5),
])
def test_bad_input_rejected_before_device(case, status):
    st, h = _create(**case)
    assert st == status, spc5.lib().spc5_last_error()
    assert h.value is None   # *out is cleared on failure
    assert spc5.lib().spc5_last_error()


@needs_lib
def test_null_out_and_null_handles():
    L = spc5.lib()
    st, _ = _create([0, 1], [0], [1.0], 1, 3, out=False)
    assert st == -1
    assert L.spc5_spmv(None, None, None, None) == -1
    assert L.spc5_spmv_noalloc(None, None, None, None) == -1
    assert L.spc5_spmv_transpose(None, None, None, None) == -1
    assert L.spc5_get_info(None, None) == -1
    assert L.spc5_to_csr(None, None, None, None) == -1
    assert L.spc5_set_variant(None, 1) == -1
    assert L.spc5_prepare_transpose(None, 0, 0) == -1
    assert L.spc5_csr_spmv(None, None, None, None) == -1
    L.spc5_free(None)
    L.spc5_csr_free(None)
    L.spc5_batch_free(None)


@needs_lib
def test_csr_create_rejects_bad_input():
    L = spc5.lib()
    h = ctypes.c_void_p(7)
    rp = np.array([0, 2], np.int64)
    ci = np.array([1, 0], np.int32)
    va = np.array([1.0, 2.0])
    st = L.spc5_csr_create(1, 3, spc5._np_ptr(rp), spc5._np_ptr(ci), spc5._np_ptr(va), 0,
                           ctypes.byref(h))
    assert st == -2 and h.value is None
