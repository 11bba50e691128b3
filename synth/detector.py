"""Synthetic Upstream Tracker description: geometry, field model and hit resolution.

The paper describes four planar strip layers (UTaX, UTaU, UTbV, UTbX) with vertical strips in the X
layers and +5 / -5 degree stereo strips in U and V (Section III-A), a hit decoded to "X at Y=0" plus
its Z, a y-range and a weight (Section IV), and a magnetic kick taken from field look-up tables
(Section III-C).  The real geometry and field maps are not public, so this module builds a uniform
stand-in: S sectors of 512 strips at 0.19 mm pitch per layer, side by side in x, and a single-kick
field model.  Every number the reconstruction needs is exported here as float32, once, so that the
reconstruction (oracle or GPU) reads the same detector description.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_LAYERS = 4
STRIPS_PER_SECTOR = 512
FRAC_BITS = 3                      # 1/8-strip interstrip fraction
PITCH_MM = 0.19
SECTOR_WIDTH_MM = STRIPS_PER_SECTOR * PITCH_MM   # 97.28 mm
Z_LAYERS_MM = (2330.0, 2380.0, 2600.0, 2650.0)
STEREO_DEG = (0.0, 5.0, -5.0, 0.0)
Z_VELO_MM = 770.0                  # z of the VELO state
K_KICK_MM_MEV = 1.2e3              # single-kick strength: delta(tx) = K * (q/p) / lever
Z_KICK_MM = 770.0                  # kink position of the single-kick model
L_LEVER_MM = 1720.0                # z_mid(UT) - z_kick = 2490 - 770
Y_HALF_MM = 650.0                  # planes are about 1.3 m high
SIGMA0_MM = 0.05                   # resolution of a one-strip cluster


@dataclass(frozen=True)
class Detector:
    """Float32 description of the synthetic UT, as the reconstruction consumes it.

    u0[l*S + s] is the measured coordinate (x at y=0) of the centre of the first 1/8-strip bin of
    sector s in layer l; a hit with strip i and fraction f sits at u0 + (8*i + f) * pitch8.
    a_kick[l] is the x deflection at layer l per unit of q/p (mm*MeV), the field table of this
    single-kick model.
    """
    n_sectors: int
    z_layer: np.ndarray            # f32[4]
    dxdy: np.ndarray               # f32[4], tan(stereo angle); x = u + y*dxdy
    a_kick: np.ndarray             # f32[4]
    u0: np.ndarray                 # f32[4*S]
    z_velo: np.float32
    pitch8: np.float32
    u_min: np.float32
    sector_width: np.float32
    inv_sector_width: np.float32
    y_begin: np.float32
    y_end: np.float32
    weight_by_size: np.ndarray     # f32[16]; index = cluster size, [0] unused (padding word)
    n_layers: int = N_LAYERS
    # float64 physics used only by the simulation
    u_min_f64: float = field(default=0.0)

    @property
    def n_banks_per_event(self) -> int:
        return self.n_layers * self.n_sectors


def make_detector(n_sectors: int) -> Detector:
    if n_sectors <= 0 or n_sectors % 2:
        raise ValueError("n_sectors must be a positive even number")
    S = n_sectors
    u_min = -S * SECTOR_WIDTH_MM / 2.0
    s = np.arange(S, dtype=np.float64)
    u0_one = (u_min + s * SECTOR_WIDTH_MM + PITCH_MM / 16.0).astype(np.float32)
    u0 = np.tile(u0_one, N_LAYERS)
    z = np.array(Z_LAYERS_MM, dtype=np.float32)
    dxdy = np.array([math.tan(math.radians(a)) for a in STEREO_DEG], dtype=np.float32)
    a_kick = np.array([K_KICK_MM_MEV * (zz - Z_KICK_MM) / L_LEVER_MM for zz in Z_LAYERS_MM],
                      dtype=np.float32)
    w = np.zeros(16, dtype=np.float32)
    for size in range(1, 16):
        sigma = SIGMA0_MM * (1.0 + 0.25 * (size - 1))
        w[size] = np.float32(1.0 / (sigma * sigma))
    return Detector(
        n_sectors=S, z_layer=z, dxdy=dxdy, a_kick=a_kick, u0=u0,
        z_velo=np.float32(Z_VELO_MM), pitch8=np.float32(PITCH_MM / 8.0),
        u_min=np.float32(u_min), sector_width=np.float32(SECTOR_WIDTH_MM),
        inv_sector_width=np.float32(1.0 / SECTOR_WIDTH_MM),
        y_begin=np.float32(-Y_HALF_MM), y_end=np.float32(Y_HALF_MM),
        weight_by_size=w, u_min_f64=u_min)


@dataclass(frozen=True)
class CompassParams:
    """Algorithm knobs of the tracklet search (Section V), all float32 / int32.

    Window half-width W = w0 + kw / p_min (mm).  max_hits is the per-layer window cap (the
    "number of hit candidates"), n_sectors_search the 1/3/5 sector choice (Section V-A).
    slope_tol bounds |t_pair - tx_velo|; completion_tol widens the completion interval (mm).
    max_tracklets 0 selects the minimum over every compatible combination; N > 0 the paper's
    search (closest completion hit per layer, stop after N tracklets, Section V-B).
    """
    w0: np.float32
    kw: np.float32
    p_min: np.float32
    max_hits: int
    n_sectors_search: int
    slope_tol: np.float32
    completion_tol: np.float32
    max_tracklets: int = 0


def make_compass_params(p_min_mev: float = 1500.0, max_hits: int = 8, n_sectors_search: int = 5,
                        w0_mm: float = 0.5, kw_mm_mev: float = 1500.0,
                        completion_tol_mm: float = 0.5, max_tracklets: int = 0) -> CompassParams:
    # The pair slope differs from the VELO slope by at most the kick K/(p_min*lever), plus the
    # resolution term 2*eps over the anchor lever arm of 270 mm.
    slope_tol = K_KICK_MM_MEV / (p_min_mev * L_LEVER_MM) + 2.0 * completion_tol_mm / 270.0
    return CompassParams(
        w0=np.float32(w0_mm), kw=np.float32(kw_mm_mev), p_min=np.float32(p_min_mev),
        max_hits=int(max_hits), n_sectors_search=int(n_sectors_search),
        slope_tol=np.float32(slope_tol), completion_tol=np.float32(completion_tol_mm),
        max_tracklets=int(max_tracklets))
