"""Thin ctypes binding of libutcompass.so (include/ut_compass.h).

Argument marshalling only: torch provides device memory and the stream; every step of decoding,
window search, tracklet finding, fitting and the adjoint runs in the library's HIP kernels.  The
binding fails loudly when the library is not built or when no GPU is present; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

from .build import LIB

_f = ctypes.c_float
_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t

FLAG_BANK_ORDER = 1
FLAG_CAPACITY = 2
FLAG_LAYER_OVERFLOW = 4
FLAG_BANK_SIZE = 8
MAX_BANK_WORDS = 8192
NOALLOC_MAX_EVENTS = 32768


class UtcGeometry(ctypes.Structure):
    _fields_ = [("n_layers", _i32), ("n_sectors", _i32), ("z_layer", _f * 4), ("dxdy", _f * 4),
                ("a_kick", _f * 4), ("z_velo", _f), ("pitch8", _f), ("u_min", _f),
                ("sector_width", _f), ("inv_sector_width", _f), ("y_begin", _f), ("y_end", _f),
                ("weight_by_size", _f * 16), ("u0", _P)]


class UtcCompassParams(ctypes.Structure):
    _fields_ = [("w0", _f), ("kw", _f), ("p_min", _f), ("max_hits", _i32),
                ("n_sectors_search", _i32), ("slope_tol", _f), ("completion_tol", _f),
                ("max_tracklets", _i32)]


class UtcLaunchConfig(ctypes.Structure):
    _fields_ = [("block", _i32), ("grid", _i32), ("window_tile", _i32), ("reserved", _i32)]


_lib = None


def library():
    """Load libutcompass.so (built in-tree by paper_2002_11529_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built; run `python -m paper_2002_11529_amd.build`")
    L = ctypes.CDLL(LIB)
    L.ut_decode_workspace_bytes.restype = _sz
    L.ut_decode_workspace_bytes.argtypes = [_i32, _i32]
    L.ut_decode.restype = ctypes.c_int
    L.ut_decode.argtypes = [_P, _P, _P, _i32, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _sz, _P, _P]
    L.ut_decode_noalloc.restype = ctypes.c_int
    L.ut_decode_noalloc.argtypes = [_P, _P, _P, _i32, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.compass_find_workspace_bytes.restype = _sz
    L.compass_find_workspace_bytes.argtypes = [_i32, _i64]
    L.compass_find.restype = ctypes.c_int
    L.compass_find.argtypes = [_P, _P, _i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _i64,
                               _P, _P, _P, _P, _P, _P, _P, _sz, _P, _P]
    L.compass_fit_grad_workspace_bytes.restype = _sz
    L.compass_fit_grad_workspace_bytes.argtypes = [_i32]
    L.compass_fit_grad.restype = ctypes.c_int
    L.compass_fit_grad.argtypes = [_P, _i64, _P, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _f, _P,
                                   _P, _P, _P, _P, _sz, _P]
    L.compass_fit_freeze.restype = ctypes.c_int
    L.compass_fit_freeze.argtypes = [_P, _i64, _P, _i64, _P, _P, _P, _P, _P, _P, _P]
    L.compass_fit_grad_frozen.restype = ctypes.c_int
    L.compass_fit_grad_frozen.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _f, _P, _P,
                                          _P, _P, _P, _sz, _P]
    for name in ("ut_decode_autotune", "compass_find_autotune"):
        getattr(L, name).restype = ctypes.c_int
    L.ut_decode_autotune.argtypes = [_P, _P, _P, _i32, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                     _sz, _i32, _P, _P, _P]
    L.compass_find_autotune.argtypes = [_P, _P, _i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        _i64, _P, _P, _P, _P, _P, _P, _sz, _i32, _P, _P, _P]
    L.utc_status_string.restype = ctypes.c_char_p
    L.utc_status_string.argtypes = [ctypes.c_int]
    L.utc_version.restype = ctypes.c_char_p
    L.ut_global_event_cut_workspace_bytes.restype = _sz
    L.ut_global_event_cut_workspace_bytes.argtypes = [_i32]
    L.ut_global_event_cut.restype = ctypes.c_int
    L.ut_global_event_cut.argtypes = [_P, _i32, _P, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P, _P, _P,
                                      _P, _P, _P, _P, _P, _P, _P, _P, _sz, _P]
    L.compass_consolidate_workspace_bytes.restype = _sz
    L.compass_consolidate_workspace_bytes.argtypes = [_i64]
    L.compass_consolidate.restype = ctypes.c_int
    L.compass_consolidate.argtypes = [_i32, _P, _i64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                      _sz, _P]
    _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        msg = library().utc_status_string(status).decode()
        raise RuntimeError(f"{what} failed: {msg} ({status})")


# element kinds the C ABI expects: (bytes per element, floating point)
_KINDS = {"i16": (2, False), "i32": (4, False), "f32": (4, True), "f64": (8, True)}


def _ptr(t: Optional[torch.Tensor], kind: Optional[str] = None):
    """Device pointer of a contiguous tensor (None passes NULL); with `kind`, the element width and
    type are checked, since the library reads raw memory."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if kind is not None:
        size, fp = _KINDS[kind]
        if t.element_size() != size or t.is_floating_point() != fp:
            raise ValueError(f"{kind} tensor expected, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _launch(launch):
    if launch is None:
        return None
    c = UtcLaunchConfig()
    c.block = int(launch.get("block", 256))
    c.grid = int(launch.get("grid", 0))
    c.window_tile = int(launch.get("tile", 0))
    return ctypes.byref(c)


class Geometry:
    """Detector description for the library: float32 scalars plus the device u0 table."""

    def __init__(self, det, device="cuda"):
        self.n_sectors = int(det.n_sectors)
        self.u0 = torch.as_tensor(det.u0, dtype=torch.float32).to(device).contiguous()
        s = UtcGeometry()
        s.n_layers = 4
        s.n_sectors = self.n_sectors
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
        s.u0 = self.u0.data_ptr()
        self.struct = s

    @property
    def ref(self):
        return ctypes.byref(self.struct)


def compass_params(p) -> UtcCompassParams:
    s = UtcCompassParams()
    s.w0, s.kw, s.p_min = float(p.w0), float(p.kw), float(p.p_min)
    s.max_hits, s.n_sectors_search = int(p.max_hits), int(p.n_sectors_search)
    s.slope_tol, s.completion_tol = float(p.slope_tol), float(p.completion_tol)
    s.max_tracklets = int(getattr(p, "max_tracklets", 0))
    return s


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def ut_decode(geom: Geometry, words, bank_offsets, n_events: int, hit_capacity: Optional[int] = None,
              error_flags=None, launch=None, out=None, workspace=None, stream=None, compact=False):
    """Decode raw banks into the hit structure of arrays.  Returns a dict of device tensors.
    compact=True leaves out the layer / geometry constants z, y_begin and y_end."""
    L = library()
    dev = words.device
    n_banks = n_events * 4 * geom.n_sectors
    if bank_offsets.shape[0] != n_banks + 1:
        raise ValueError("bank_offsets must have n_events*4*S + 1 entries")
    cap = int(words.shape[0]) if hit_capacity is None else int(hit_capacity)
    if out is None:
        out = dict(hit_offsets=torch.empty(n_banks + 1, dtype=torch.int32, device=dev),
                   lhcbid=torch.empty(cap, dtype=torch.int32, device=dev),
                   u=torch.empty(cap, dtype=torch.float32, device=dev),
                   weight=torch.empty(cap, dtype=torch.float32, device=dev))
        if not compact:
            for k in ("z", "y_begin", "y_end"):
                out[k] = torch.empty(cap, dtype=torch.float32, device=dev)
    if error_flags is None:
        error_flags = torch.zeros(1, dtype=torch.int32, device=dev)
    out["error_flags"] = error_flags
    if workspace is None:
        workspace = _workspace(L.ut_decode_workspace_bytes(n_events, geom.n_sectors), dev)
    st = L.ut_decode(geom.ref, _ptr(words, "i16"), _ptr(bank_offsets, "i32"), n_events, cap,
                     _ptr(out["hit_offsets"], "i32"), _ptr(out["lhcbid"], "i32"),
                     _ptr(out.get("z"), "f32"), _ptr(out["u"], "f32"),
                     _ptr(out.get("y_begin"), "f32"), _ptr(out.get("y_end"), "f32"),
                     _ptr(out["weight"], "f32"), _ptr(error_flags, "i32"), _ptr(workspace),
                     workspace.numel(), _launch(launch), _stream(stream))
    _check(st, "ut_decode")
    return out


def ut_decode_noalloc(geom: Geometry, words, bank_offsets, n_events: int, out,
                      hit_capacity: Optional[int] = None, error_flags=None, launch=None, stream=None):
    """ut_decode through the entry point that allocates nothing: the caller passes every output
    (`out`, a dict of device tensors as ut_decode returns it, and `error_flags`); the library's
    fixed per-GPU scratch array replaces the workspace.  Calls on one GPU must not overlap."""
    L = library()
    n_banks = n_events * 4 * geom.n_sectors
    if bank_offsets.shape[0] != n_banks + 1:
        raise ValueError("bank_offsets must have n_events*4*S + 1 entries")
    if error_flags is None:
        raise ValueError("error_flags must be passed (this entry point allocates nothing)")
    cap = int(words.shape[0]) if hit_capacity is None else int(hit_capacity)
    st = L.ut_decode_noalloc(geom.ref, _ptr(words, "i16"), _ptr(bank_offsets, "i32"), n_events, cap,
                             _ptr(out["hit_offsets"], "i32"), _ptr(out["lhcbid"], "i32"),
                             _ptr(out.get("z"), "f32"), _ptr(out["u"], "f32"),
                             _ptr(out.get("y_begin"), "f32"), _ptr(out.get("y_end"), "f32"),
                             _ptr(out["weight"], "f32"), _ptr(error_flags, "i32"), _launch(launch),
                             _stream(stream))
    _check(st, "ut_decode_noalloc")
    return out


def compass_find(geom: Geometry, params, n_events: int, hits, vx, vy, vtx, vty, velo_offsets,
                 windows: bool = False, error_flags=None, launch=None, out=None, workspace=None,
                 stream=None, n_tracks=None):
    """Compass tracklet search for every VELO track.  Returns a dict of device tensors."""
    L = library()
    dev = vx.device
    n = int(vx.shape[0]) if n_tracks is None else int(n_tracks)
    if out is None:
        out = dict(hit_idx=torch.empty((n, 4), dtype=torch.int32, device=dev),
                   qop=torch.empty(n, dtype=torch.float32, device=dev),
                   chi2=torch.empty(n, dtype=torch.float32, device=dev),
                   nhits=torch.empty(n, dtype=torch.int32, device=dev))
        if windows:
            out["windows"] = torch.empty((n, 4, 2), dtype=torch.int16, device=dev)
    if error_flags is None:
        error_flags = hits.get("error_flags") if isinstance(hits, dict) else None
        if error_flags is None:
            error_flags = torch.zeros(1, dtype=torch.int32, device=dev)
    out["error_flags"] = error_flags
    if workspace is None:
        workspace = _workspace(L.compass_find_workspace_bytes(n_events, n), dev)
    p = params if isinstance(params, UtcCompassParams) else compass_params(params)
    st = L.compass_find(geom.ref, ctypes.byref(p), n_events, _ptr(hits["hit_offsets"], "i32"),
                        _ptr(hits["u"], "f32"), _ptr(hits["weight"], "f32"),
                        _ptr(hits.get("y_begin"), "f32"), _ptr(hits.get("y_end"), "f32"),
                        _ptr(vx, "f32"), _ptr(vy, "f32"), _ptr(vtx, "f32"), _ptr(vty, "f32"),
                        _ptr(velo_offsets, "i32"), n, _ptr(out["hit_idx"], "i32"),
                        _ptr(out["qop"], "f32"), _ptr(out["chi2"], "f32"), _ptr(out["nhits"], "i32"),
                        _ptr(out.get("windows"), "i16"), _ptr(error_flags, "i32"), _ptr(workspace),
                        workspace.numel(), _launch(launch), _stream(stream))
    _check(st, "compass_find")
    return out


def compass_fit_grad(geom: Geometry, track_hit_idx, hit_u, hit_weight, hit_lhcbid, vx, vy, vtx, vty,
                     qop, offsets, grad_scale: float = 1.0, want_grad: bool = True,
                     want_chi2_track: bool = True, out=None, workspace=None, stream=None):
    """Chi2 of the frozen track fits and (optionally) its gradients.  Returns a dict of tensors."""
    L = library()
    dev = qop.device
    n = int(qop.shape[0])
    S = geom.n_sectors
    if out is None:
        out = dict(chi2_total=torch.empty(1, dtype=torch.float64, device=dev))
        if want_chi2_track:
            out["chi2_track"] = torch.empty(n, dtype=torch.float32, device=dev)
        if want_grad:
            out["grad_qop"] = torch.empty(n, dtype=torch.float32, device=dev)
            out["grad_offsets"] = torch.empty(4 * S, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(L.compass_fit_grad_workspace_bytes(S), dev)
    st = L.compass_fit_grad(geom.ref, n, _ptr(track_hit_idx, "i32"), int(hit_u.shape[0]),
                            _ptr(hit_u, "f32"), _ptr(hit_weight, "f32"), _ptr(hit_lhcbid, "i32"),
                            _ptr(vx, "f32"), _ptr(vy, "f32"), _ptr(vtx, "f32"), _ptr(vty, "f32"),
                            _ptr(qop, "f32"), _ptr(offsets, "f32"), float(grad_scale),
                            _ptr(out.get("chi2_track"), "f32"), _ptr(out.get("chi2_total"), "f64"),
                            _ptr(out.get("grad_qop"), "f32"), _ptr(out.get("grad_offsets"), "f32"),
                            _ptr(workspace), workspace.numel(), _stream(stream))
    _check(st, "compass_fit_grad")
    return out


def _fit_grad_workspace(geom: Geometry, device):
    """One fit-gradient workspace per geometry and device, kept on the Geometry object and reused by
    every call made through CompassChi2Function (calls on one stream only; the workspace is
    scratch of a single call)."""
    cache = geom.__dict__.setdefault("_fit_grad_ws", {})
    key = str(torch.device(device))
    if key not in cache:
        cache[key] = _workspace(library().compass_fit_grad_workspace_bytes(geom.n_sectors), device)
    return cache[key]


def compass_fit_freeze(geom: Geometry, track_hit_idx, hit_u, hit_weight, hit_lhcbid, out=None,
                       stream=None):
    """The frozen hits of the fits in track-major form (u, weight, global sector per layer).
    Returns dict(track_u, track_weight, track_sector) of shape (n, 4)."""
    L = library()
    dev = hit_u.device
    n = int(track_hit_idx.shape[0])
    if out is None:
        out = dict(track_u=torch.empty((n, 4), dtype=torch.float32, device=dev),
                   track_weight=torch.empty((n, 4), dtype=torch.float32, device=dev),
                   track_sector=torch.empty((n, 4), dtype=torch.int16, device=dev))
    st = L.compass_fit_freeze(geom.ref, n, _ptr(track_hit_idx, "i32"), int(hit_u.shape[0]),
                              _ptr(hit_u, "f32"), _ptr(hit_weight, "f32"), _ptr(hit_lhcbid, "i32"),
                              _ptr(out["track_u"], "f32"), _ptr(out["track_weight"], "f32"),
                              _ptr(out["track_sector"], "i16"), _stream(stream))
    _check(st, "compass_fit_freeze")
    return out


def compass_fit_grad_frozen(geom: Geometry, frozen, vx, vy, vtx, vty, qop, offsets,
                            grad_scale: float = 1.0, want_grad: bool = True,
                            want_chi2_track: bool = True, out=None, workspace=None, stream=None):
    """compass_fit_grad on hits frozen by compass_fit_freeze (same results)."""
    L = library()
    dev = qop.device
    n = int(qop.shape[0])
    S = geom.n_sectors
    if out is None:
        out = dict(chi2_total=torch.empty(1, dtype=torch.float64, device=dev))
        if want_chi2_track:
            out["chi2_track"] = torch.empty(n, dtype=torch.float32, device=dev)
        if want_grad:
            out["grad_qop"] = torch.empty(n, dtype=torch.float32, device=dev)
            out["grad_offsets"] = torch.empty(4 * S, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = _workspace(L.compass_fit_grad_workspace_bytes(S), dev)
    st = L.compass_fit_grad_frozen(geom.ref, n, _ptr(frozen["track_u"], "f32"),
                                   _ptr(frozen["track_weight"], "f32"),
                                   _ptr(frozen["track_sector"], "i16"), _ptr(vx, "f32"),
                                   _ptr(vy, "f32"), _ptr(vtx, "f32"), _ptr(vty, "f32"),
                                   _ptr(qop, "f32"), _ptr(offsets, "f32"), float(grad_scale),
                                   _ptr(out.get("chi2_track"), "f32"),
                                   _ptr(out.get("chi2_total"), "f64"),
                                   _ptr(out.get("grad_qop"), "f32"),
                                   _ptr(out.get("grad_offsets"), "f32"), _ptr(workspace),
                                   workspace.numel(), _stream(stream))
    _check(st, "compass_fit_grad_frozen")
    return out


class CompassChi2Function(torch.autograd.Function):
    """chi2_total(qop, offsets) of frozen track fits, with the library's hand-written adjoint.

    Usage: chi2 = CompassChi2Function.apply(qop, offsets, geom, frozen) where `frozen` is a dict of
    device tensors track_hit_idx, hit_u, hit_weight, hit_lhcbid, vx, vy, vtx, vty.  The forward and
    backward calls share one workspace per geometry and device, so calls on several streams at once
    must not use one Geometry.
    """

    @staticmethod
    def forward(ctx, qop, offsets, geom, frozen):
        r = compass_fit_grad(geom, frozen["track_hit_idx"], frozen["hit_u"], frozen["hit_weight"],
                             frozen["hit_lhcbid"], frozen["vx"], frozen["vy"], frozen["vtx"],
                             frozen["vty"], qop.detach().contiguous(), offsets.detach().contiguous(),
                             want_grad=False, want_chi2_track=False,
                             workspace=_fit_grad_workspace(geom, qop.device))
        ctx.save_for_backward(qop, offsets)
        ctx.geom, ctx.frozen = geom, frozen
        return r["chi2_total"][0]

    @staticmethod
    def backward(ctx, grad_out):
        qop, offsets = ctx.saved_tensors
        f = ctx.frozen
        r = compass_fit_grad(ctx.geom, f["track_hit_idx"], f["hit_u"], f["hit_weight"],
                             f["hit_lhcbid"], f["vx"], f["vy"], f["vtx"], f["vty"],
                             qop.detach().contiguous(), offsets.detach().contiguous(),
                             grad_scale=1.0, want_grad=True, want_chi2_track=False,
                             workspace=_fit_grad_workspace(ctx.geom, qop.device))
        g = grad_out.to(torch.float32)
        return r["grad_qop"] * g, r["grad_offsets"] * g, None, None


def per_event_loop(geom: Geometry, params, n_events: int, words, bank_offsets, vx, vy, vtx, vty,
                   velo_offsets, host_bank_offsets, host_hit_offsets, hits_out, res_out,
                   scratch=None, stream=None):
    """The same decode + Compass work launched one event at a time (the comparison baseline of
    the batched launch).  Argument marshalling only: event e's banks are a slice of
    bank_offsets (absolute word offsets), its hits go to hits_out at the event's first hit (taken
    from host_hit_offsets of an earlier batched decode), its tracks' outputs to res_out at their
    global positions.  Hit indices in res_out come out relative to the event's first hit."""
    L = library()
    dev = words.device
    nb = 4 * geom.n_sectors
    p = params if isinstance(params, UtcCompassParams) else compass_params(params)
    if scratch is None:
        scratch = dict(hoff=torch.empty(nb + 1, dtype=torch.int32, device=dev),
                       wsd=_workspace(L.ut_decode_workspace_bytes(1, geom.n_sectors), dev),
                       wsf=_workspace(L.compass_find_workspace_bytes(1, int(vx.shape[0])), dev),
                       flags=torch.zeros(1, dtype=torch.int32, device=dev))
    n_tracks = int(vx.shape[0])
    for e in range(n_events):
        base = int(host_hit_offsets[e * nb])
        n_words = int(host_bank_offsets[(e + 1) * nb]) - int(host_bank_offsets[e * nb])
        ev_hits = {k: hits_out[k][base:] for k in ("lhcbid", "z", "u", "y_begin", "y_end", "weight")}
        ev_hits["hit_offsets"] = scratch["hoff"]
        ut_decode(geom, words, bank_offsets[e * nb:(e + 1) * nb + 1], 1,
                  hit_capacity=max(n_words, 0), error_flags=scratch["flags"], out=ev_hits,
                  workspace=scratch["wsd"], stream=stream)
        compass_find(geom, p, 1, ev_hits, vx, vy, vtx, vty, velo_offsets[e:e + 2],
                     error_flags=scratch["flags"], out=res_out, workspace=scratch["wsf"],
                     stream=stream, n_tracks=n_tracks)
    return scratch


def _cache_path():
    return os.environ.get("UTC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "utcompass", "autotune.json"))


def autotune(geom: Geometry, params, n_events: int, words, bank_offsets, vx, vy, vtx, vty,
             velo_offsets, reps: int = 5, use_cache: bool = True, stream=None):
    """Pick the launch shapes of ut_decode and compass_find for this workload shape by timing them
    in the library (ut_decode_autotune / compass_find_autotune).  The choice is cached as JSON,
    keyed by GPU architecture and workload shape.  Returns dict(decode=..., find=..., *_us)."""
    import json
    L = library()
    dev = words.device
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    p = params if isinstance(params, UtcCompassParams) else compass_params(params)
    n_tracks = int(vx.shape[0])
    key = (f"{arch}|tile|S={geom.n_sectors}|M={p.max_hits}|sec={p.n_sectors_search}|E={n_events}|"
           f"Nw={int(words.shape[0]) >> 16}|Nt={n_tracks >> 10}")
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    hits = ut_decode(geom, words, bank_offsets, n_events, stream=stream)
    ws = _workspace(L.ut_decode_workspace_bytes(n_events, geom.n_sectors), dev)
    best, best_us = UtcLaunchConfig(), ctypes.c_float()
    st = L.ut_decode_autotune(geom.ref, _ptr(words, "i16"), _ptr(bank_offsets, "i32"), n_events,
                              int(words.shape[0]), _ptr(hits["hit_offsets"], "i32"),
                              _ptr(hits["lhcbid"], "i32"), _ptr(hits["z"], "f32"), _ptr(hits["u"], "f32"),
                              _ptr(hits["y_begin"], "f32"), _ptr(hits["y_end"], "f32"),
                              _ptr(hits["weight"], "f32"), _ptr(hits["error_flags"], "i32"),
                              _ptr(ws), ws.numel(), reps, ctypes.byref(best), ctypes.byref(best_us),
                              _stream(stream))
    _check(st, "ut_decode_autotune")
    dec = dict(block=best.block, grid=best.grid, tile=best.window_tile)
    dec_us = float(best_us.value)
    res = compass_find(geom, p, n_events, hits, vx, vy, vtx, vty, velo_offsets, stream=stream)
    wsf = _workspace(L.compass_find_workspace_bytes(n_events, n_tracks), dev)
    st = L.compass_find_autotune(geom.ref, ctypes.byref(p), n_events, _ptr(hits["hit_offsets"], "i32"),
                                 _ptr(hits["u"], "f32"), _ptr(hits["weight"], "f32"),
                                 _ptr(hits["y_begin"], "f32"), _ptr(hits["y_end"], "f32"),
                                 _ptr(vx, "f32"), _ptr(vy, "f32"), _ptr(vtx, "f32"), _ptr(vty, "f32"),
                                 _ptr(velo_offsets, "i32"), n_tracks, _ptr(res["hit_idx"], "i32"),
                                 _ptr(res["qop"], "f32"), _ptr(res["chi2"], "f32"), _ptr(res["nhits"], "i32"),
                                 _ptr(res["error_flags"], "i32"),
                                 _ptr(wsf), wsf.numel(), reps, ctypes.byref(best),
                                 ctypes.byref(best_us), _stream(stream))
    _check(st, "compass_find_autotune")
    out = dict(decode=dec, decode_us=dec_us,
               find=dict(block=best.block, grid=best.grid, tile=best.window_tile),
               find_us=float(best_us.value))
    if use_cache:
        cache[key] = out
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".{os.getpid()}.tmp"
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return out


def ut_global_event_cut(geom: Geometry, n_events: int, words, bank_offsets, vx, vy, vtx, vty,
                        velo_offsets, max_words: int, error_flags=None, out=None, workspace=None,
                        stream=None):
    """The global event cut: a batch of the same n_events events in which the events with more than
    max_words raw words are empty.  Returns a dict of device tensors (words, bank_offsets, vx, vy,
    vtx, vty, velo_offsets, keep, n_kept, error_flags)."""
    L = library()
    dev = bank_offsets.device
    if out is None:
        out = dict(words=torch.empty_like(words), bank_offsets=torch.empty_like(bank_offsets),
                   vx=torch.empty_like(vx), vy=torch.empty_like(vy), vtx=torch.empty_like(vtx),
                   vty=torch.empty_like(vty), velo_offsets=torch.empty_like(velo_offsets),
                   keep=torch.empty(max(n_events, 1), dtype=torch.uint8, device=dev),
                   n_kept=torch.empty(1, dtype=torch.int32, device=dev))
    if error_flags is None:
        error_flags = torch.zeros(1, dtype=torch.int32, device=dev)
    out["error_flags"] = error_flags
    if workspace is None:
        workspace = _workspace(L.ut_global_event_cut_workspace_bytes(n_events), dev)
    st = L.ut_global_event_cut(geom.ref, n_events, _ptr(words, "i16"), _ptr(bank_offsets, "i32"),
                               _ptr(vx, "f32"), _ptr(vy, "f32"), _ptr(vtx, "f32"), _ptr(vty, "f32"),
                               _ptr(velo_offsets, "i32"), int(max_words), _ptr(out["words"], "i16"),
                               _ptr(out["bank_offsets"], "i32"), _ptr(out["vx"], "f32"),
                               _ptr(out["vy"], "f32"), _ptr(out["vtx"], "f32"), _ptr(out["vty"], "f32"),
                               _ptr(out["velo_offsets"], "i32"), _ptr(out.get("keep")),
                               _ptr(out.get("n_kept"), "i32"), _ptr(error_flags, "i32"), _ptr(workspace),
                               workspace.numel(), _stream(stream))
    _check(st, "ut_global_event_cut")
    return out


def compass_consolidate(n_events: int, velo_offsets, res, out=None, workspace=None, stream=None):
    """The found upstream tracks (nhits > 0) of compass_find's output `res`, in VELO order, in a
    dense container with per-event offsets.  Returns a dict of device tensors (offsets, velo,
    hit_idx, qop, chi2, nhits, n_found); only the first n_found rows are meaningful."""
    L = library()
    n = int(res["nhits"].shape[0])
    dev = res["nhits"].device
    if out is None:
        out = dict(offsets=torch.empty(n_events + 1, dtype=torch.int32, device=dev),
                   velo=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                   hit_idx=torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev),
                   qop=torch.empty(max(n, 1), dtype=torch.float32, device=dev),
                   chi2=torch.empty(max(n, 1), dtype=torch.float32, device=dev),
                   nhits=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                   n_found=torch.empty(1, dtype=torch.int32, device=dev))
    if workspace is None:
        workspace = _workspace(L.compass_consolidate_workspace_bytes(n), dev)
    st = L.compass_consolidate(n_events, _ptr(velo_offsets, "i32"), n, _ptr(res["nhits"], "i32"),
                               _ptr(res["hit_idx"], "i32"), _ptr(res["qop"], "f32"), _ptr(res["chi2"], "f32"),
                               _ptr(out["offsets"], "i32"), _ptr(out["velo"], "i32"),
                               _ptr(out["hit_idx"], "i32"), _ptr(out["qop"], "f32"), _ptr(out["chi2"], "f32"),
                               _ptr(out["nhits"], "i32"), _ptr(out.get("n_found"), "i32"), _ptr(workspace),
                               workspace.numel(), _stream(stream))
    _check(st, "compass_consolidate")
    return out


def version() -> str:
    return library().utc_version().decode()
