"""Python access to the plain CPU oracle (oracle.c) through ctypes.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the CPU-baseline leg of
the benchmark, never by the product package.  It shares no code with the GPU library; it only reads
the same synthetic detector description and events.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

FLAG_BANK_ORDER = 1
FLAG_CAPACITY = 2
FLAG_LAYER_OVERFLOW = 4
FLAG_BANK_SIZE = 8
MAX_BANK_WORDS = 8192

_f = ctypes.c_float
_P = ctypes.c_void_p


class OraDetector(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("n_sectors", ctypes.c_int32),
                ("z_layer", _f * 4), ("dxdy", _f * 4), ("a_kick", _f * 4),
                ("z_velo", _f), ("pitch8", _f), ("u_min", _f), ("sector_width", _f),
                ("inv_sector_width", _f), ("y_begin", _f), ("y_end", _f),
                ("weight_by_size", _f * 16), ("u0", _P)]


class OraParams(ctypes.Structure):
    _fields_ = [("w0", _f), ("kw", _f), ("p_min", _f), ("max_hits", ctypes.c_int32),
                ("n_sectors_search", ctypes.c_int32), ("slope_tol", _f), ("completion_tol", _f),
                ("max_tracklets", ctypes.c_int32)]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no GPU code)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.ora_ut_decode.restype = ctypes.c_int
        L.ora_compass_find.restype = ctypes.c_int
        L.ora_fit_grad_f32.restype = ctypes.c_double
        L.ora_fit_grad_f64.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def make_detector_struct(det):
    """Fill the oracle's own detector struct from a synthetic detector description."""
    u0 = np.ascontiguousarray(det.u0, dtype=np.float32)
    s = OraDetector()
    s.n_layers = det.n_layers
    s.n_sectors = det.n_sectors
    for i in range(4):
        s.z_layer[i] = float(det.z_layer[i])
        s.dxdy[i] = float(det.dxdy[i])
        s.a_kick[i] = float(det.a_kick[i])
    s.z_velo = float(det.z_velo)
    s.pitch8 = float(det.pitch8)
    s.u_min = float(det.u_min)
    s.sector_width = float(det.sector_width)
    s.inv_sector_width = float(det.inv_sector_width)
    s.y_begin = float(det.y_begin)
    s.y_end = float(det.y_end)
    for i in range(16):
        s.weight_by_size[i] = float(det.weight_by_size[i])
    s.u0 = u0.ctypes.data_as(_P)
    return s, u0


def make_params_struct(p):
    s = OraParams()
    s.w0, s.kw, s.p_min = float(p.w0), float(p.kw), float(p.p_min)
    s.max_hits, s.n_sectors_search = int(p.max_hits), int(p.n_sectors_search)
    s.slope_tol, s.completion_tol = float(p.slope_tol), float(p.completion_tol)
    s.max_tracklets = int(getattr(p, "max_tracklets", 0))
    return s


def decode(det, words, bank_offsets, n_events, hit_capacity=None):
    """Run the oracle decoder.  Returns a dict of numpy arrays plus 'flags'."""
    words = np.ascontiguousarray(words, dtype=np.uint16)
    bank_offsets = np.ascontiguousarray(bank_offsets, dtype=np.uint32)
    n_banks = n_events * det.n_layers * det.n_sectors
    if bank_offsets.shape[0] != n_banks + 1:
        raise ValueError("bank_offsets must have E*L*S+1 entries")
    cap = int(np.count_nonzero(words & 0xF)) if hit_capacity is None else int(hit_capacity)
    out = dict(hit_offsets=np.zeros(n_banks + 1, np.uint32), lhcbid=np.zeros(cap, np.uint32),
               z=np.zeros(cap, np.float32), u=np.zeros(cap, np.float32),
               y_begin=np.zeros(cap, np.float32), y_end=np.zeros(cap, np.float32),
               weight=np.zeros(cap, np.float32))
    ds, keep = make_detector_struct(det)
    rc = lib().ora_ut_decode(ctypes.byref(ds), _ptr(words), _ptr(bank_offsets),
                             ctypes.c_int32(n_events), ctypes.c_int64(cap),
                             _ptr(out["hit_offsets"]), _ptr(out["lhcbid"]), _ptr(out["z"]),
                             _ptr(out["u"]), _ptr(out["y_begin"]), _ptr(out["y_end"]),
                             _ptr(out["weight"]))
    if rc < 0:
        raise ValueError(f"oracle decode rejected its arguments ({rc})")
    out["flags"] = rc
    return out


def compass(det, params, n_events, hits, velo_x, velo_y, velo_tx, velo_ty, velo_offsets,
            with_windows=False):
    """Run the oracle tracklet search on decoded hits (a dict as returned by decode())."""
    vx = np.ascontiguousarray(velo_x, np.float32)
    vy = np.ascontiguousarray(velo_y, np.float32)
    vtx = np.ascontiguousarray(velo_tx, np.float32)
    vty = np.ascontiguousarray(velo_ty, np.float32)
    vo = np.ascontiguousarray(velo_offsets, np.uint32)
    n = int(vx.shape[0])
    out = dict(hit_idx=np.zeros((n, 4), np.int32), qop=np.zeros(n, np.float32),
               chi2=np.zeros(n, np.float32), nhits=np.zeros(n, np.int32))
    if with_windows:
        out.update(win_first=np.zeros((n, 4), np.int32), win_size=np.zeros((n, 4), np.int32),
                   active=np.zeros(n, np.uint8))
    ds, keep = make_detector_struct(det)
    ps = make_params_struct(params)
    arrs = [np.ascontiguousarray(hits[k]) for k in ("hit_offsets", "u", "weight", "y_begin", "y_end")]
    rc = lib().ora_compass_find(
        ctypes.byref(ds), ctypes.byref(ps), ctypes.c_int32(n_events),
        *[_ptr(a) for a in arrs], _ptr(vx), _ptr(vy), _ptr(vtx), _ptr(vty), _ptr(vo),
        _ptr(out["hit_idx"]), _ptr(out["qop"]), _ptr(out["chi2"]), _ptr(out["nhits"]),
        _ptr(out.get("win_first")), _ptr(out.get("win_size")), _ptr(out.get("active")))
    if rc < 0:
        raise ValueError(f"oracle compass rejected its arguments ({rc})")
    out["flags"] = rc
    return out


def fit_grad(det, track_hit_idx, hit_u, hit_weight, hit_lhcbid, velo_x, velo_y, velo_tx, velo_ty,
             qop, offsets, grad_scale=1.0, precision="f32"):
    """Chi2 per track, total, and gradients w.r.t. qop and the per-sector offsets."""
    dt = np.float32 if precision == "f32" else np.float64
    idx = np.ascontiguousarray(track_hit_idx, np.int32)
    n = int(idx.shape[0])
    qop = np.ascontiguousarray(qop, dt)
    offsets = np.ascontiguousarray(offsets, dt)
    c2 = np.zeros(n, dt)
    gq = np.zeros(n, dt)
    go = np.zeros(4 * det.n_sectors, dt)
    ds, keep = make_detector_struct(det)
    args = [ctypes.byref(ds), ctypes.c_int64(n), _ptr(idx), ctypes.c_int64(int(np.shape(hit_u)[0])),
            _ptr(np.ascontiguousarray(hit_u, np.float32)),
            _ptr(np.ascontiguousarray(hit_weight, np.float32)),
            _ptr(np.ascontiguousarray(hit_lhcbid, np.uint32)),
            _ptr(np.ascontiguousarray(velo_x, np.float32)), _ptr(np.ascontiguousarray(velo_y, np.float32)),
            _ptr(np.ascontiguousarray(velo_tx, np.float32)), _ptr(np.ascontiguousarray(velo_ty, np.float32)),
            _ptr(qop), _ptr(offsets)]
    if precision == "f32":
        total = lib().ora_fit_grad_f32(*args, ctypes.c_float(grad_scale), _ptr(c2), _ptr(gq), _ptr(go))
    else:
        total = lib().ora_fit_grad_f64(*args, ctypes.c_double(grad_scale), _ptr(c2), _ptr(gq), _ptr(go))
    return dict(chi2_total=float(total), chi2_track=c2, grad_qop=gq, grad_offsets=go)
