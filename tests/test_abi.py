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


def test_python_option_names_match_the_header():
    """Every tuning option of the binding has the value its BCG_OPT_ constant has."""
    from paper_1710_09745_amd import bcg
    text = open(HEADER).read()
    enum = dict((k.lower(), int(v)) for k, v in re.findall(r"\bBCG_OPT_([A-Z_]+)\s*=\s*(\d+)", text))
    count = enum.pop("count")
    assert bcg.OPTIONS == enum
    assert sorted(enum.values()) == list(range(count))


def test_float_reciprocal_row_index_is_exact():
    """The N x N kernels take e / N as trunc((e + 1/2) * rcp(N)) in float32 for
    1 <= N <= 64 and 0 <= e < 65 N; the hardware reciprocal is within one ulp of
    1/N, and every one of the three nearest float32 values gives the exact
    quotient (the float32 products round as the kernel's do)."""
    import numpy as np
    for n in range(1, 65):
        r0 = np.float32(1.0) / np.float32(n)
        e = np.arange(65 * n, dtype=np.int64)
        for r in (np.nextafter(r0, np.float32(0)), r0, np.nextafter(r0, np.float32(1))):
            q = ((e.astype(np.float32) + np.float32(0.5)) * np.float32(r)).astype(np.int64)
            assert np.array_equal(q, e // n), n
