"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/cm.h, and rejects invalid arguments
before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2110_00853_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "cm.h")).read()
    return sorted(set(re.findall(r"CM_API\s+[\w\s\*]+?\b(cm_\w+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in declared():
        assert hasattr(L, name), name


def test_invalid_grid_arguments_are_rejected_on_the_host():
    L = B.load()
    out = C.c_void_p()
    d = B.GridDesc()
    d.N = 5
    for a in range(3):
        d.ne[a] = 2
        d.lo[a] = 0.0
        d.hi[a] = 1.0
    assert L.cm_grid_create(C.byref(d), 0, C.byref(out)) == B.CM_ERR_UNSUPPORTED
    d.N = 4
    d.ne[1] = 0
    assert L.cm_grid_create(C.byref(d), 0, C.byref(out)) == B.CM_ERR_ARG
    assert b"ne >= 1" in L.cm_last_error()
    assert L.cm_grid_create(None, 0, C.byref(out)) == B.CM_ERR_ARG
    assert L.cm_dg_rhs(None, None, None, 0.0, None) == B.CM_ERR_ARG
    assert L.cm_lsrk_step(None, None, None, None, 0.0, 1.0, None) == B.CM_ERR_ARG
    assert L.cm_model_create(None, None, None, C.byref(out)) == B.CM_ERR_ARG


def test_grid_beyond_32_bit_indexing_is_rejected_on_the_host():
    """The kernels index nodes x words in 32-bit integers: a mesh whose node
    count times 16 words reaches 2^31 is refused before any device call."""
    L = B.load()
    out = C.c_void_p()
    d = B.GridDesc()
    d.N = 4
    for a in range(3):
        d.ne[a] = 256
        d.lo[a] = 0.0
        d.hi[a] = 1.0
    assert L.cm_grid_create(C.byref(d), 0, C.byref(out)) == B.CM_ERR_UNSUPPORTED
    assert b"32-bit" in L.cm_last_error()
    assert not out.value

