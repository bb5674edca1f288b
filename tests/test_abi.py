"""CPU checks of the C-ABI library: it loads, exports every function that
include/spamm.h declares, and argument checks that touch no device answer
without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1906_08148_amd import spamm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "spamm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(spamm_[a-z_]+)\s*\(", text))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(spamm.LIB_PATH):
        pytest.fail("libspamm.so not built: run __graft_entry__.build()")
    return spamm.load_library()


def test_every_declared_symbol_is_exported(lib):
    decl = declared_functions()
    assert len(decl) >= 15
    for name in sorted(decl):
        assert hasattr(lib, name), name
    assert decl == set(spamm._SIGS), "binding and header disagree"


def test_status_strings(lib):
    for code, name in spamm.STATUS.items():
        assert lib.spamm_status_string(code).decode() == "SPAMM_" + name


def test_ctx_create_rejects_bad_arguments(lib):
    out = ctypes.c_void_p()
    # NULL arena / tiny arena / misaligned arena are refused before any HIP call
    assert lib.spamm_ctx_create(0, None, 1 << 30, None, ctypes.byref(out)) == 1
    assert lib.spamm_ctx_create(0, ctypes.c_void_p(4096), 1024, None, ctypes.byref(out)) == 1
    assert lib.spamm_ctx_create(0, ctypes.c_void_p(4096 + 8), 1 << 30, None, ctypes.byref(out)) == 1
    assert lib.spamm_ctx_create(0, ctypes.c_void_p(4096), 1 << 30, None, None) == 1


def test_null_handles_are_rejected(lib):
    assert lib.spamm_release(None, None) == 0
    info = spamm.MatInfo()
    assert lib.spamm_mat_info_get(None, ctypes.byref(info)) == 1
    assert lib.spamm_ctx_destroy(None) == 1
    out = ctypes.c_void_p()
    d = ctypes.c_double()
    for fn in (lib.spamm_truncate, lib.spamm_truncate_symmetric, lib.spamm_truncate_elementwise):
        assert fn(None, None, 1.0, ctypes.byref(out), ctypes.byref(d)) == 1  # EINVAL, no context
        assert fn(None, None, 1.0, None, None) == 1
