"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/hodlr.h, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HDR = os.path.join(ROOT, "include", "hodlr.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hodlr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2208_06290_amd import hodlr
    if not os.path.exists(hodlr.LIB_PATH):
        pytest.fail("libhodlr.so is not built (run __graft_entry__.build())")
    return hodlr.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("hodlr_factor", "hodlr_solve", "hodlr_solve_adjoint", "hodlr_matvec", "hodlr_grad"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2208_06290_amd import hodlr
    assert set(hodlr.EXPORTS) == set(_declared())


def test_status_strings(lib):
    for code, txt in ((0, b"ok"), (-1, b"invalid argument"), (1, b"exactly singular pivot")):
        assert lib.hodlr_status_string(code) == txt


def _mat(n=64, levels=1, ranks=(4,), offsets=None, dtype=0, ld=None):
    from paper_2208_06290_amd import hodlr
    m = hodlr._Matrix()
    m.n = n
    m.levels = levels
    r = (ctypes.c_int32 * max(1, len(ranks)))(*ranks)
    m.ranks = r
    if offsets is not None:
        off = (ctypes.c_int64 * len(offsets))(*offsets)
        m.leaf_offsets = off
    else:
        off = None
    m.dtype = dtype
    m.D = m.U = m.V = 0x1000  # never dereferenced: validation fails first
    m.ldd = m.ldu = m.ldv = n if ld is None else ld
    return m, (r, off)


@pytest.mark.parametrize("kw", [
    dict(n=0),
    dict(levels=-1),
    dict(n=64, levels=7, ranks=(1,) * 7),      # 2^L > N
    dict(n=63, levels=1),                       # not divisible, no offsets
    dict(offsets=(0, 40, 30)),                  # not increasing
    dict(offsets=(0, 32, 65)),                  # does not end at N
    dict(ranks=(-1,)),
    dict(ld=10),                                # leading dimension < N
    dict(dtype=7),
    dict(n=64, levels=1, ranks=(33,)),          # r_1 = 33 > 32 rows per level-1 node
    dict(n=64, levels=2, ranks=(4, 17)),        # r_2 = 17 > 16 rows per level-2 node
    dict(offsets=(0, 3, 64), ranks=(4,)),       # a 3-row node cannot hold rank 4
])
def test_bad_arguments_are_rejected_before_launch(lib, kw):
    from paper_2208_06290_amd import hodlr
    m, keep = _mat(**kw)
    h = ctypes.c_void_p()
    st = lib.hodlr_factor(ctypes.byref(m), 0, 0, None, ctypes.byref(h), None)
    assert st == -1 and not h


def test_limits_are_reported_as_unsupported(lib):
    m, keep = _mat(n=1024, levels=1, ranks=(65,))
    h = ctypes.c_void_p()
    assert lib.hodlr_factor(ctypes.byref(m), 0, 0, None, ctypes.byref(h), None) == -4
    m, keep = _mat(n=1024, levels=1, ranks=(4,))  # leaves of 512 > HODLR_MAX_LEAF
    assert lib.hodlr_factor(ctypes.byref(m), 0, 0, None, ctypes.byref(h), None) == -4
    m, keep = _mat(n=64, levels=1, ranks=(4,), dtype=1)  # FP64 factor of FP32 storage
    assert lib.hodlr_factor(ctypes.byref(m), 0, 0, None, ctypes.byref(h), None) == -4


def test_flags_are_checked(lib):
    h = ctypes.c_void_p()
    m, keep = _mat(n=64, levels=1, ranks=(4,))
    assert lib.hodlr_factor(ctypes.byref(m), 0, 2, None, ctypes.byref(h), None) == -1   # unknown flag bit
    m, keep = _mat(n=200, levels=0, ranks=())
    assert lib.hodlr_factor(ctypes.byref(m), 0, 1, None, ctypes.byref(h), None) == -4   # in place: 200 % 16 != 0
    m, keep = _mat(n=64, levels=1, ranks=(4,), dtype=0)
    assert lib.hodlr_factor(ctypes.byref(m), 1, 1, None, ctypes.byref(h), None) == -4   # in place: F32 factors of F64 D
    assert not h


def _cpu(*shape, dtype=None):
    import torch
    return torch.zeros(*shape, dtype=dtype or torch.float64)


@pytest.mark.parametrize("bad", ["U_rows", "V_rows", "D_rows", "offsets_len", "strided_N", "dtype_mix"])
def test_python_matrix_shapes_are_checked_before_any_device_use(bad):
    import torch
    from paper_2208_06290_amd import hodlr
    n, ranks = 256, [4, 4]
    D, U, V = _cpu(64, n), _cpu(8, n), _cpu(8, n)
    off = None
    if bad == "U_rows":
        U = _cpu(7, n)
    elif bad == "V_rows":
        V = _cpu(9, n)
    elif bad == "D_rows":
        D = _cpu(63, n)
    elif bad == "offsets_len":
        off = [0, 64, 128, 256]
    elif bad == "strided_N":
        U = _cpu(8, 2 * n)[:, ::2]
    else:
        V = _cpu(8, n, dtype=torch.float32)
    with pytest.raises(ValueError) as e:
        hodlr.HODLRMatrix(D, U, V, ranks, off)
    assert "device" not in str(e.value)


def test_python_matrix_with_valid_shapes_needs_device_tensors():
    from paper_2208_06290_amd import hodlr
    with pytest.raises(ValueError, match="device"):
        hodlr.HODLRMatrix(_cpu(64, 256), _cpu(8, 256), _cpu(8, 256), [4, 4])


def test_null_solve_arguments(lib):
    assert lib.hodlr_solve(None, 1, None, 1, None, None, None) == -1
    assert lib.hodlr_solve_adjoint(None, 1, None, 1, None, None, None) == -1
    assert lib.hodlr_grad(None, 1, None, 1, None, 1, None, None, None, None) == -1
