"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function include/bcg.h declares, and argument errors are reported
without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcg.h")
LIB = os.path.join(ROOT, "paper_1710_09745_amd", "libbcg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["bcg_create", "bcg_destroy", "bcg_load_links", "bcg_set_mass", "bcg_set_solver",
              "bcg_apply", "bcg_hop", "bcg_solve", "bcg_solve_cg", "bcg_link_force",
              "bcg_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbcg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbcg.so not built")
def test_create_rejects_bad_dims_without_a_device():
    from paper_1710_09745_amd import bcg
    lib = bcg.load_library()
    h = ctypes.c_void_p()
    for dims in [(4, 4, 4, 5), (4, 0, 4, 4), (1, 4, 4, 4)]:
        rc = lib.bcg_create(ctypes.byref(h), (ctypes.c_int * 4)(*dims), 1, None)
        assert rc == bcg.ERR_ARG
        assert b"even" in lib.bcg_last_error(None)
    rc = lib.bcg_create(ctypes.byref(h), (ctypes.c_int * 4)(4, 4, 4, 4), 2, None)
    assert rc == bcg.ERR_ARG
    assert lib.bcg_create(None, (ctypes.c_int * 4)(4, 4, 4, 4), 1, None) == bcg.ERR_ARG
