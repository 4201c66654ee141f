"""The C ABI loads and exports every symbol that include/kifmm.h declares;
argument errors come back as status codes (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kifmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kifmm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2512_09478_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2512_09478_amd import build
        build.build()
    return _lib.lib()


def test_header_symbols_exported(L):
    names = declared_functions()
    assert "kifmm_setup" in names and "kifmm_backward" in names and "kifmm_clump_reduce" in names
    for n in names:
        assert hasattr(L, n), n
    from paper_2512_09478_amd import _lib
    assert sorted(_lib.EXPORTS) == names


def test_argument_errors_without_gpu(L):
    h = ctypes.c_void_p()
    # null positions
    assert L.kifmm_setup(None, 10, 0, 4, 8, ctypes.byref(h)) == -1
    assert h.value is None
    msg = L.kifmm_status_string(-1).decode()
    assert "invalid argument" in msg and "positions" in msg
    dummy = ctypes.c_void_p(16)      # never dereferenced: the checks fail first
    assert L.kifmm_setup(dummy, 0, 0, 4, 8, ctypes.byref(h)) == -1          # N < 1
    assert L.kifmm_setup(dummy, 10, 7, 4, 8, ctypes.byref(h)) == -1         # kernel
    assert L.kifmm_setup(dummy, 10, 0, 1, 8, ctypes.byref(h)) == -1         # p < 2
    assert L.kifmm_setup(dummy, 10, 0, 9, 8, ctypes.byref(h)) == -1         # p > 8
    assert L.kifmm_setup(dummy, 10, 0, 4, 0, ctypes.byref(h)) == -1         # leaf < 1
    from paper_2512_09478_amd._lib import Options
    o = Options()
    L.kifmm_default_options(ctypes.byref(o))
    assert o.adaptive == 1 and o.max_depth == 21 and o.pinv_rtol == 1e-7
    o.max_depth = 22
    assert L.kifmm_setup_ex(dummy, 10, 0, 4, 8, ctypes.byref(o), None, ctypes.byref(h)) == -1
    L.kifmm_default_options(ctypes.byref(o))
    o.explicit_root = 1
    o.root_side = 3.0
    assert L.kifmm_setup_ex(dummy, 10, 0, 4, 8, ctypes.byref(o), None, ctypes.byref(h)) == -1
    o.root_side = 1.0
    o.root_lo[0] = 1e-5             # not on the side/4096 grid
    assert L.kifmm_setup_ex(dummy, 10, 0, 4, 8, ctypes.byref(o), None, ctypes.byref(h)) == -1
    # null handles
    assert L.kifmm_evaluate(None, dummy, None, None, None) == -5
    assert L.kifmm_evaluate_dipoles(None, dummy, dummy, None, None, None) == -5
    assert L.kifmm_evaluate_gradient(None, dummy, None, None, None, None, None) == -5
    assert L.kifmm_backward(None, dummy, None, None, None, None, None) == -5
    assert L.kifmm_clump_reduce(None, dummy, dummy, dummy, 1, dummy, dummy, dummy, None) == -5
    assert L.kifmm_clump_backward(None, dummy, dummy, dummy, 1, dummy, None, None, None, None, None, None,
                                  None) == -5
    out = (ctypes.c_int64 * 10)()
    assert L.kifmm_get_counts(None, out) == -5
    assert L.kifmm_get_m2l_rank(None, out) == -5
    L.kifmm_destroy(None)
