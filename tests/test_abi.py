"""The C-ABI library: it loads, exports every entry point its header declares, and rejects bad
arguments on the host without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ut_compass.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\*?\s+\**(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_11529_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("ut_decode", "compass_find", "compass_fit_grad", "ut_decode_workspace_bytes",
              "compass_find_workspace_bytes", "compass_fit_grad_workspace_bytes",
              "utc_status_string", "utc_version"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_version_and_status_strings(lib):
    lib.utc_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.utc_version()
    lib.utc_status_string.restype = ctypes.c_char_p
    assert lib.utc_status_string(0) == b"ok"
    assert lib.utc_status_string(-2).startswith(b"workspace")


def test_workspace_sizes(lib):
    lib.ut_decode_workspace_bytes.restype = ctypes.c_size_t
    lib.ut_decode_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert lib.ut_decode_workspace_bytes(1000, 200) >= (2 * 4000 + 1) * 4
    assert lib.ut_decode_workspace_bytes(1000, 200) % 256 == 0
    lib.compass_fit_grad_workspace_bytes.restype = ctypes.c_size_t
    lib.compass_fit_grad_workspace_bytes.argtypes = [ctypes.c_int32]
    assert lib.compass_fit_grad_workspace_bytes(200) >= 2 * 801 * 8


def test_host_argument_errors_return_without_launching():
    """NULL geometry / negative sizes / bad params are rejected on the host (no GPU needed)."""
    import numpy as np
    import synth
    import paper_2002_11529_amd.api as api
    L = api.library()
    assert L.ut_decode(None, None, None, 1, 0, None, None, None, None, None, None, None, None,
                       None, 0, None, None) == -1
    det = synth.make_detector(32)
    g = api.UtcGeometry()
    g.n_layers, g.n_sectors, g.u0 = 4, 32, 16  # a non-NULL placeholder; never dereferenced here
    # negative event count
    assert L.ut_decode(ctypes.byref(g), None, None, -1, 0, None, None, None, None, None, None, None,
                       None, None, 0, None, None) == -1
    # workspace missing
    one = ctypes.c_void_p(64)
    assert L.ut_decode(ctypes.byref(g), one, one, 1, 10, one, one, one, one, one, one, one, None,
                       None, 0, None, None) == -2
    p = api.compass_params(synth.make_compass_params())
    p.max_hits = 33
    assert L.compass_find(ctypes.byref(g), ctypes.byref(p), 1, one, one, one, one, one, one, one,
                          one, one, one, 1, one, one, one, one, None, None, one, 256, None,
                          None) == -1
    p.max_hits, p.n_sectors_search = 8, 4
    assert L.compass_find(ctypes.byref(g), ctypes.byref(p), 1, one, one, one, one, one, one, one,
                          one, one, one, 1, one, one, one, one, None, None, one, 256, None,
                          None) == -1
    assert L.compass_fit_grad(ctypes.byref(g), -1, None, 0, None, None, None, None, None, None,
                              None, None, None, 1.0, None, None, None, None, None, 0, None) == -1
