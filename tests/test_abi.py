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


def test_host_checks_of_every_entry_point():
    """Launch-shape limits, the pointer rules of the compact hit form, parameter ranges and workspace
    sizes are checked on the host before anything is enqueued (none of these calls reaches the GPU;
    placeholder pointers are never dereferenced)."""
    import synth
    import paper_2002_11529_amd.api as api
    L = api.library()
    g = api.UtcGeometry()
    g.n_layers, g.n_sectors, g.u0 = 4, 32, 16
    one = ctypes.c_void_p(64)
    ws_dec = L.ut_decode_workspace_bytes(1, 32)

    def decode(launch=None, z=one, yb=one, ye=one, ws=None, ws_bytes=0, n_events=1):
        return L.ut_decode(ctypes.byref(g), one, one, n_events, 10, one, one, z, one, yb, ye, one, None,
                           ws, ws_bytes, ctypes.byref(launch) if launch else None, None)

    # the compact form: z, y_begin, y_end may be NULL (the call gets as far as the workspace check)
    assert decode(z=None, yb=None, ye=None) == -2
    # launch shapes: block a multiple of 64 in [64, 1024]
    for block, ok in ((32, False), (96, False), (1088, False), (64, True), (1024, True)):
        lc = api.UtcLaunchConfig()
        lc.block, lc.grid = block, 0
        assert decode(launch=lc) == (-2 if ok else -1), block
    lc = api.UtcLaunchConfig()
    lc.block, lc.grid = 256, -1
    assert decode(launch=lc) == -1
    # window tile: 0 (default) or 4 .. 40 KiB per wavefront
    for tile, ok in ((-1, False), (1, False), (3, False), (0, True), (4, True), (40, True), (41, False)):
        lc = api.UtcLaunchConfig()
        lc.block, lc.grid, lc.window_tile = 256, 0, tile
        assert decode(launch=lc) == (-2 if ok else -1), tile
    # workspace one byte short
    assert decode(ws=one, ws_bytes=ws_dec - 1) == -2

    p = api.compass_params(synth.make_compass_params())

    def find(launch=None, yb=one, ye=one, ws=one, ws_bytes=256, n_tracks=1, n_events=1):
        return L.compass_find(ctypes.byref(g), ctypes.byref(p), n_events, one, one, one, yb, ye, one,
                              one, one, one, one, n_tracks, one, one, one, one, None, None, ws,
                              ws_bytes, ctypes.byref(launch) if launch else None, None)

    # nothing to do: returns ok without launching
    assert find(n_tracks=0) == 0 and find(n_events=0) == 0
    # per-hit y ranges: both or neither
    assert find(n_tracks=0, yb=None, ye=None) == 0
    assert find(yb=None) == -1 and find(ye=None) == -1
    assert find(ws=None) == -2 and find(ws_bytes=8) == -2
    for block, ok in ((576, False), (1024, False), (512, True), (64, True)):
        lc = api.UtcLaunchConfig()
        lc.block, lc.grid = block, 0
        assert (find(launch=lc, n_tracks=0) == 0) == ok, block
    for tile, ok in ((-1, False), (2, False), (0, True), (4, True), (40, True), (41, False)):
        lc = api.UtcLaunchConfig()
        lc.block, lc.grid, lc.window_tile = 256, 0, tile
        assert (find(launch=lc, n_tracks=0) == 0) == ok, tile
    for field, bad in (("max_hits", 0), ("max_hits", 33), ("n_sectors_search", 2), ("max_tracklets", -1)):
        q = api.compass_params(synth.make_compass_params())
        setattr(q, field, bad)
        assert L.compass_find(ctypes.byref(g), ctypes.byref(q), 1, one, one, one, one, one, one, one,
                              one, one, one, 0, one, one, one, one, None, None, one, 256, None,
                              None) == -1, field

    # fit gradient: workspace sized for the geometry
    need = L.compass_fit_grad_workspace_bytes(32)
    args = [ctypes.byref(g), 1, one, 4, one, one, one, one, one, one, one, one, one, 1.0, one, one, one,
            one]
    assert L.compass_fit_grad(*args, one, need - 1, None) == -2
    assert L.compass_fit_grad(*args, None, need, None) == -2
    bad = list(args)
    bad[2] = None                      # track_hit_idx missing
    assert L.compass_fit_grad(*bad, one, need, None) == -1

    # global event cut and consolidation
    cut_ws = L.ut_global_event_cut_workspace_bytes(3)
    cut = lambda n_events, ws, ws_bytes, words=one: L.ut_global_event_cut(
        ctypes.byref(g), n_events, words, one, one, one, one, one, one, 100, one, one, one, one, one, one,
        one, one, one, None, ws, ws_bytes, None)
    assert cut(-1, one, cut_ws) == -1
    assert cut(3, one, cut_ws, words=None) == -1
    assert cut(3, one, cut_ws - 1) == -2
    cons_ws = L.compass_consolidate_workspace_bytes(10)
    cons = lambda n_tracks, ws_bytes, nhits=one: L.compass_consolidate(
        2, one, n_tracks, nhits, one, one, one, one, one, one, one, one, one, one, one, ws_bytes, None)
    assert cons(-1, cons_ws) == -1
    assert cons(10, cons_ws, nhits=None) == -1
    assert cons(10, cons_ws - 1) == -2


def test_noalloc_decode_rejects_on_the_host():
    """ut_decode_noalloc checks its arguments, and the event count against its fixed scratch,
    before it touches a GPU."""
    import paper_2002_11529_amd.api as api
    L = api.library()
    g = api.UtcGeometry()
    g.n_layers, g.n_sectors, g.u0 = 4, 32, 16  # a non-NULL placeholder; never dereferenced here
    one = ctypes.c_void_p(64)
    assert L.ut_decode_noalloc(None, one, one, 1, 10, one, one, one, one, one, one, one, None,
                               None, None) == -1
    assert L.ut_decode_noalloc(ctypes.byref(g), one, one, -1, 10, one, one, one, one, one, one,
                               one, None, None, None) == -1
    assert L.ut_decode_noalloc(ctypes.byref(g), one, one, api.NOALLOC_MAX_EVENTS + 1, 10, one,
                               one, one, one, one, one, one, None, None, None) == -1
