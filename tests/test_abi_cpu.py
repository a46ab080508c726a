"""The C ABI library loads and exports what include/mdlj.h declares; the
argument checks that run before any device call behave as documented.
No GPU is needed: nothing here launches a kernel or allocates device memory."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = ""
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text += open(os.path.join(ROOT, "include", fn)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdlj_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def m():
    from paper_2512_03565_amd import mdlj
    return mdlj


def test_library_exports_every_declared_symbol(m):
    syms = declared_symbols()
    assert len(syms) >= 25
    missing = [s for s in syms if not hasattr(m.lib, s)]
    assert not missing, missing


def test_version(m):
    assert "gfx950" in m.version()


def test_create_rejects_bad_arguments_before_device_work(m):
    x = np.zeros(4)
    p = x.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    assert m.lib.mdlj_create(None, 4, p, p, p, None, 1, 0, None) == -1
    assert m.lib.mdlj_create(C.byref(h), 0, p, p, p, None, 1, 0, None) == -1
    assert m.lib.mdlj_create(C.byref(h), 4, None, p, p, None, 1, 0, None) == -1
    assert m.lib.mdlj_create(C.byref(h), 4, p, p, p, None, 0, 0, None) == -1
    assert m.lib.mdlj_create(C.byref(h), 4, p, p, p, None, 9, 0, None) == -1
    assert m.lib.mdlj_create(C.byref(h), 4, p, p, p, None, 1, 7, None) == -1
    bad = np.array([0.0, np.nan, 1.0, 2.0])
    assert m.lib.mdlj_create(C.byref(h), 4, bad.ctypes.data_as(C.c_void_p), p, p, None, 1, 0,
                             None) == -6
    t = np.array([0, 1, 2, 0], np.int32)
    assert m.lib.mdlj_create(C.byref(h), 4, p, p, p, t.ctypes.data_as(C.c_void_p), 2, 0,
                             None) == -1
    assert not h.value


def test_null_context_is_rejected(m):
    assert m.lib.mdlj_destroy(None) == 0
    assert m.lib.mdlj_set_box(None, 1.0, 1.0, 1.0) == -1
    assert m.lib.mdlj_set_cutoff(None, 1.0) == -1
    assert m.lib.mdlj_compute_forces(None, None, None, None, 0, None, None) == -1
    assert m.lib.mdlj_tune(None, 0, 1, None, None) == -1
    n = C.c_int32()
    assert m.lib.mdlj_config_count(None, C.byref(n)) == -1
    assert m.lib.mdlj_last_error(None) == b"null context"


def test_index_views_reject_bad_arguments(m):
    i32 = C.POINTER(C.c_int32)
    cell = np.empty(4, np.int32)
    nc = np.empty(3, np.int32)
    assert m.lib.mdlj_get_cells(None, cell.ctypes.data_as(i32), nc.ctypes.data_as(i32)) == -1
    cnt = C.c_int64()
    assert m.lib.mdlj_get_pairs(None, 0, None, None, C.byref(cnt)) == -1
