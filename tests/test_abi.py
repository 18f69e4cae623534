"""CPU-side checks of the C ABI: the library loads, exports every function
that include/rsg.h declares, and rejects bad arguments before touching the
GPU.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsg.h")
LIB = os.path.join(ROOT, "paper_1501_05654_amd", "librsg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1501_05654_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["rsg_grid_create", "rsg_ham_create", "rsg_hpsi", "rsg_propagate_step",
              "rsg_propagate", "rsg_dot", "rsg_norm2", "rsg_energy", "rsg_adjoint_step",
              "rsg_control_forward", "rsg_control_backward", "rsg_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_argument_errors(lib):
    lib.rsg_last_error.restype = C.c_char_p
    lib.rsg_grid_create.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    out = C.c_void_p()
    assert lib.rsg_grid_create(None, None, C.byref(out)) == -1
    assert b"null" in lib.rsg_last_error()

    class Desc(C.Structure):
        _fields_ = [("shape", C.c_int32), ("n", C.c_int32), ("radius", C.c_double), ("h", C.c_double)]

    assert lib.rsg_grid_create(C.byref(Desc(7, 4, 0.0, 0.3)), None, C.byref(out)) == -1
    assert b"shape" in lib.rsg_last_error()
    assert lib.rsg_grid_create(C.byref(Desc(0, 4, 0.0, -1.0)), None, C.byref(out)) == -1
    assert lib.rsg_grid_create(C.byref(Desc(1, 0, -2.0, 0.3)), None, C.byref(out)) == -1
    assert lib.rsg_grid_create(C.byref(Desc(0, 0, 0.0, 0.3)), None, C.byref(out)) == -1
    lib.rsg_hpsi.argtypes = [C.c_void_p] * 3 + [C.c_int64, C.c_int64, C.c_int32, C.c_double,
                                                C.c_void_p, C.c_size_t, C.c_void_p]
    assert lib.rsg_hpsi(None, None, None, 1, 1, 0, 0.0, None, 0, None) == -1
    lib.rsg_laser_field.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int64,
                                    C.c_int64, C.c_void_p, C.c_void_p]
    assert lib.rsg_laser_field(None, 3, 1.0, 0.1, 0, 4, None, None) == -1
    lib.rsg_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    assert lib.rsg_copy(None, None, 15, None) == -1
    lib.rsg_version.restype = C.c_char_p
    assert b"gfx950" in lib.rsg_version()


def test_row_alignment_argument_errors(lib):
    lib.rsg_last_error.restype = C.c_char_p

    class Desc(C.Structure):
        _fields_ = [("shape", C.c_int32), ("n", C.c_int32), ("radius", C.c_double), ("h", C.c_double)]

    lib.rsg_grid_create_aligned.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    out = C.c_void_p()
    for align in (0, -8, 3, 12, 128):
        assert lib.rsg_grid_create_aligned(C.byref(Desc(0, 8, 0.0, 0.3)), align, None, C.byref(out)) == -1
        assert b"align" in lib.rsg_last_error()
    assert lib.rsg_grid_create_aligned(None, 8, None, C.byref(out)) == -1
    assert b"null" in lib.rsg_last_error()


def test_box_grid_and_noalloc_argument_errors(lib):
    """Rectangular boxes and the allocation-free inner product reject bad
    arguments on the host, before any device call."""
    lib.rsg_last_error.restype = C.c_char_p
    lib.rsg_grid_create_box.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_void_p,
                                        C.c_void_p]
    out = C.c_void_p()
    assert lib.rsg_grid_create_box(8, 8, 8, 0.3, 1, None, None) == -1
    assert b"null" in lib.rsg_last_error()
    for nx, ny, nz in ((0, 4, 4), (4, -1, 4), (4, 4, 0)):
        assert lib.rsg_grid_create_box(nx, ny, nz, 0.3, 1, None, C.byref(out)) == -1
        assert b"at least 1 point" in lib.rsg_last_error()
    assert lib.rsg_grid_create_box(40000, 1, 1, 0.3, 1, None, C.byref(out)) == -1
    assert b"32767" in lib.rsg_last_error()
    assert lib.rsg_grid_create_box(4, 4, 4, 0.0, 1, None, C.byref(out)) == -1
    assert b"h must be" in lib.rsg_last_error()
    assert lib.rsg_grid_create_box(4, 4, 4, 0.3, 3, None, C.byref(out)) == -1
    assert b"align" in lib.rsg_last_error()
    lib.rsg_dot_noalloc_max_bytes.restype = C.c_size_t
    assert lib.rsg_dot_noalloc_max_bytes() == 1 << 20
    lib.rsg_dot_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                    C.c_void_p]
    assert lib.rsg_dot_noalloc(None, None, None, 1, 1, None, None) < 0
