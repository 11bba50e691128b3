"""Seeded generator of UT raw banks plus VELO track states.

Event model (a stand-in for the LHCb minbias samples, which are not available):
  * VELO tracks: state at z = 770 mm with x, y ~ N(0, 1) mm and tx, ty ~ U(-0.25, 0.25);
    p = 3 GeV + Exp(mean 10 GeV), charge +-1 with equal probability.
  * Hidden particles: same kinematics, UT hits only, no VELO state.  They stand in for the tracks
    that leave UT hits without a matching VELO track (Section III-B).
  * A particle crosses layer l at x = x0 + tx*dz + (q/p)*a_kick[l], y = y0 + ty*dz; it leaves a hit
    with probability 0.97, measured u = x - y*dxdy smeared by N(0, 0.05 mm), quantised to 1/8 strip.
  * Noise hits: uniform over (layer, sector, strip, fraction).
  * Cluster size in {1, 2, 3} with probabilities {0.6, 0.3, 0.1}.
  * Raw bank format: one bank per (event, layer, sector), banks ordered event-major, then layer,
    then sector.  A bank is a list of uint16 words  strip<<7 | fraction<<4 | size;  size 0 marks
    a padding word.  Words inside a bank are shuffled, and every bank with an odd number of hits
    gets one padding word (so banks are 32-bit aligned) at a random position.
    bank_offsets[b] .. bank_offsets[b+1] (in words) delimit bank b.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .detector import (Detector, CompassParams, make_detector, make_compass_params,
                       N_LAYERS, SECTOR_WIDTH_MM, PITCH_MM, Y_HALF_MM, SIGMA0_MM)

HIT_EFFICIENCY = 0.97
SIZE_PROBS = (0.6, 0.3, 0.1)       # cluster sizes 1, 2, 3

# truth codes for words that are not VELO-track hits
TRUTH_NOISE = -1
TRUTH_HIDDEN = -2
TRUTH_PADDING = -3


@dataclass
class EventBatch:
    name: str
    seed: int
    detector: Detector
    params: CompassParams
    n_events: int
    words: np.ndarray              # u16[Nw]
    bank_offsets: np.ndarray       # u32[E*L*S + 1]
    velo_x: np.ndarray             # f32[Nt]
    velo_y: np.ndarray
    velo_tx: np.ndarray
    velo_ty: np.ndarray
    velo_offsets: np.ndarray       # u32[E + 1]
    qop_true: np.ndarray           # f64[Nt]
    n_layers_hit: np.ndarray       # i8[Nt], number of layers in which the VELO track left a hit
    delta_true: Optional[np.ndarray] = None   # f32[L*S] hidden per-sector x offsets (mm)
    truth: dict = field(default_factory=dict)
    outside: Optional[np.ndarray] = None      # i8[Nt] how a track was put outside the planes (OUTSIDE_*)

    @property
    def n_tracks(self) -> int:
        return int(self.velo_x.shape[0])

    @property
    def n_words(self) -> int:
        return int(self.words.shape[0])

    @property
    def n_valid_words(self) -> int:
        return int(np.count_nonzero(self.words & 0xF))


# Workload recipes: sizes and distributions of the synthetic stand-ins for the paper's samples.
CONFIGS = {
    "tiny": dict(n_sectors=32, n_events=100, seed=1, tracks=("fixed", 50),
                 noise=("fixed", 200), hidden=("none",), p_min=1500.0, max_hits=8),
    "realistic": dict(n_sectors=200, n_events=1000, seed=2, tracks=("fixed", 200),
                      noise=("poisson", 750), hidden=("poisson", 380), p_min=1500.0, max_hits=8),
    "batched": dict(n_sectors=32, n_events=20000, seed=3,
                    tracks=("lognormal", 200.0, 0.5, 10, 1500),
                    noise=("poisson", 500), hidden=("scaled", 15.0 / 3.88 - 1.0),
                    p_min=1500.0, max_hits=8),
    "fitgrad": dict(n_sectors=200, n_events=21000, seed=4, tracks=("fixed", 50),
                    noise=("fixed", 200), hidden=("none",), p_min=1500.0, max_hits=8,
                    misalign_sigma=0.1),
    "pileup": dict(n_sectors=200, n_events=10000, seed=5,
                   tracks=("lognormal", 500.0, 0.4, 50, 3000),
                   noise=("poisson", 4000), hidden=("topup", 6000.0, 3.88),
                   p_min=1000.0, max_hits=16),
}


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def _counts(rng, spec, n_events, base=None):
    kind = spec[0]
    if kind == "none":
        return np.zeros(n_events, dtype=np.int64)
    if kind == "fixed":
        return np.full(n_events, int(spec[1]), dtype=np.int64)
    if kind == "poisson":
        return rng.poisson(spec[1], size=n_events).astype(np.int64)
    if kind == "lognormal":
        median, sigma, lo, hi = spec[1:]
        v = np.rint(rng.lognormal(np.log(median), sigma, size=n_events))
        return np.clip(v, lo, hi).astype(np.int64)
    if kind == "scaled":
        return np.rint(spec[1] * base).astype(np.int64)
    if kind == "topup":
        target, per_track = spec[1:]
        return np.maximum(0, np.rint((target - per_track * base) / per_track)).astype(np.int64)
    raise ValueError(f"unknown count spec {spec}")


def _particles(rng, n):
    x = rng.normal(0.0, 1.0, n).astype(np.float32)
    y = rng.normal(0.0, 1.0, n).astype(np.float32)
    tx = rng.uniform(-0.25, 0.25, n).astype(np.float32)
    ty = rng.uniform(-0.25, 0.25, n).astype(np.float32)
    p = 3000.0 + rng.exponential(10000.0, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return x, y, tx, ty, q / p


CHUNK_EVENTS = 1024   # events are drawn in blocks with a random stream of their own

# Ways a VELO track is placed outside the planes (generator option outside_fraction): its straight
# line leaves the plane height only at the last layer, only at the first layer, or the plane width
# only at the last or only at the first layer; the other checked layer stays inside.
OUTSIDE_NONE, OUTSIDE_Y_LAST, OUTSIDE_Y_FIRST, OUTSIDE_U_LAST, OUTSIDE_U_FIRST = 0, 1, 2, 3, 4


def _place_outside(rng, det, S, vx, vy, vtx, vty, fraction):
    """Move a random `fraction` of the VELO states so that their straight line misses the planes in
    one of the four OUTSIDE_* ways (chosen uniformly); returns the per-track code."""
    n = vx.shape[0]
    code = np.where(rng.random(n) < fraction, rng.integers(1, 5, n), 0).astype(np.int8)
    dz0 = float(det.z_layer[0]) - float(det.z_velo)
    dz3 = float(det.z_layer[3]) - float(det.z_velo)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    beyond = rng.uniform(0.01, 40.0, n)      # how far past the edge (mm)
    inside = rng.uniform(5.0, 150.0, n)      # how far inside the edge at the other layer (mm)
    y_half, u_half = float(Y_HALF_MM), S * SECTOR_WIDTH_MM / 2.0
    for c, half, last in ((OUTSIDE_Y_LAST, y_half, True), (OUTSIDE_Y_FIRST, y_half, False),
                          (OUTSIDE_U_LAST, u_half, True), (OUTSIDE_U_FIRST, u_half, False)):
        m = code == c
        out_at = sign[m] * (half + beyond[m])
        in_at = sign[m] * (half - inside[m])
        at0, at3 = (in_at, out_at) if last else (out_at, in_at)
        slope = (at3 - at0) / (dz3 - dz0)
        start = at0 - slope * dz0
        if c in (OUTSIDE_Y_LAST, OUTSIDE_Y_FIRST):
            vy[m], vty[m] = start.astype(np.float32), slope.astype(np.float32)
        else:
            vx[m], vtx[m] = start.astype(np.float32), slope.astype(np.float32)
    return code


def _chunk(rng, det, E, S, tracks, noise, hidden, delta_true, extra_padding_prob, with_truth,
           outside_fraction=0.0):
    """Draw E events; event indices and track ids are local to the block."""
    L = N_LAYERS
    n_velo = _counts(rng, tracks, E)
    n_hidden = _counts(rng, hidden, E, base=n_velo)
    n_noise = _counts(rng, noise, E)

    # particles: VELO tracks (in event order) then hidden particles (in event order)
    Nv, Nh = int(n_velo.sum()), int(n_hidden.sum())
    vx, vy, vtx, vty, vqop = _particles(rng, Nv)
    hx, hy, htx, hty, hqop = _particles(rng, Nh)
    outside = (_place_outside(rng, det, S, vx, vy, vtx, vty, outside_fraction)
               if outside_fraction > 0 else np.zeros(Nv, np.int8))
    px = np.concatenate([vx, hx]).astype(np.float64)
    py = np.concatenate([vy, hy]).astype(np.float64)
    ptx = np.concatenate([vtx, htx]).astype(np.float64)
    pty = np.concatenate([vty, hty]).astype(np.float64)
    pqop = np.concatenate([vqop, hqop])
    pev = np.concatenate([np.repeat(np.arange(E, dtype=np.int32), n_velo),
                          np.repeat(np.arange(E, dtype=np.int32), n_hidden)])
    NP = Nv + Nh

    # particle x layer crossings
    dz = det.z_layer.astype(np.float64) - np.float64(det.z_velo)
    dxdy = det.dxdy.astype(np.float64)
    a = det.a_kick.astype(np.float64)
    eff = rng.random((NP, L)) < HIT_EFFICIENCY
    smear = rng.normal(0.0, SIGMA0_MM, (NP, L))
    y = py[:, None] + pty[:, None] * dz[None, :]
    u_meas = px[:, None] + ptx[:, None] * dz[None, :] + pqop[:, None] * a[None, :]
    u_meas -= y * dxdy[None, :]
    u_meas += smear
    del smear
    if delta_true is not None:
        sec_f = np.floor((u_meas - det.u_min_f64) / SECTOR_WIDTH_MM)
        sidx = np.clip(sec_f, 0, S - 1).astype(np.int64) + (np.arange(L) * S)[None, :]
        u_meas += delta_true[sidx].astype(np.float64)
    keep = eff & (np.abs(y) <= Y_HALF_MM)
    pos = u_meas - det.u_min_f64
    sec = np.floor(pos / SECTOR_WIDTH_MM)
    keep &= (sec >= 0) & (sec < S)
    pi, li = np.nonzero(keep)
    t_sec = sec[pi, li].astype(np.int32)
    within = pos[pi, li] - t_sec * SECTOR_WIDTH_MM
    t_q = np.clip(np.floor(within / (PITCH_MM / 8.0)), 0, 4095).astype(np.int32)
    n_layers_hit = np.bincount(pi[pi < Nv], minlength=Nv).astype(np.int8)

    # noise
    NN = int(n_noise.sum())
    n_layer = rng.integers(0, L, NN, dtype=np.int32)
    n_sec = rng.integers(0, S, NN, dtype=np.int32)
    n_q = rng.integers(0, 4096, NN, dtype=np.int32)

    ev = np.concatenate([pev[pi], np.repeat(np.arange(E, dtype=np.int32), n_noise)])
    layer = np.concatenate([li.astype(np.int32), n_layer])
    sector = np.concatenate([t_sec, n_sec])
    qv = np.concatenate([t_q, n_q])
    NHIT = ev.shape[0]
    size = (1 + np.searchsorted(np.cumsum(SIZE_PROBS), rng.random(NHIT), side="right")).astype(np.int32)
    size = np.minimum(size, 3)
    bank = (ev.astype(np.int64) * L + layer) * S + sector
    words = ((qv >> 3) << 7) | ((qv & 7) << 4) | size

    # padding words: one per odd bank (32-bit alignment) plus optional random extra pairs
    NB = E * L * S
    counts = np.bincount(bank, minlength=NB)
    pad_banks = np.nonzero(counts & 1)[0]
    if extra_padding_prob > 0:
        extra = np.nonzero(rng.random(NB) < extra_padding_prob)[0]
        pad_banks = np.concatenate([pad_banks, extra, extra])
    NPAD = pad_banks.shape[0]
    bank = np.concatenate([bank, pad_banks])
    words = np.concatenate([words, np.zeros(NPAD, dtype=np.int32)])

    # shuffle inside banks: sort by (bank, random 24-bit key); quicksort is deterministic for a
    # given input and much faster than a stable multi-key sort
    order = np.argsort((bank << 24) | rng.integers(0, 1 << 24, bank.shape[0]))
    counts += np.bincount(pad_banks, minlength=NB)
    out = dict(words=words[order].astype(np.uint16), bank_counts=counts, n_velo=n_velo,
               vx=vx, vy=vy, vtx=vtx, vty=vty, vqop=vqop, n_layers_hit=n_layers_hit, outside=outside)
    if with_truth:
        ptruth = np.concatenate([np.arange(Nv, dtype=np.int64), np.full(Nh, TRUTH_HIDDEN, np.int64)])
        truth_id = np.concatenate([ptruth[pi], np.full(NN, TRUTH_NOISE, np.int64),
                                   np.full(NPAD, TRUTH_PADDING, np.int64)])
        umeas = np.concatenate([u_meas[pi, li], np.full(NN + NPAD, np.nan)])
        layer = np.concatenate([layer, ((pad_banks // S) % L).astype(np.int32)])
        sector = np.concatenate([sector, (pad_banks % S).astype(np.int32)])
        qv = np.concatenate([qv, np.zeros(NPAD, dtype=np.int32)])
        size = np.concatenate([size, np.zeros(NPAD, dtype=np.int32)])
        out["truth"] = dict(track=truth_id[order], u_meas=umeas[order],
                            layer=layer[order].astype(np.int8), sector=sector[order].astype(np.int32),
                            q=qv[order].astype(np.int16), size=size[order].astype(np.int8),
                            n_hidden=n_hidden, n_noise=n_noise)
    return out


def generate(name: str = "tiny", n_events: Optional[int] = None, seed: Optional[int] = None, *,
             with_truth: bool = True, n_sectors: Optional[int] = None,
             max_hits: Optional[int] = None, n_sectors_search: int = 5,
             tracks=None, noise=None, hidden=None, misalign_sigma: Optional[float] = None,
             extra_padding_prob: float = 0.0, outside_fraction: float = 0.0) -> EventBatch:
    """Generate a batch for recipe `name`; keyword arguments override the recipe.

    outside_fraction > 0 places that fraction of the VELO tracks outside the planes at the first or
    the last layer (EventBatch.outside records how); their hits follow the moved straight lines.

    Events are drawn in blocks of CHUNK_EVENTS, block c from the stream default_rng([seed, c]);
    the per-sector offsets (when the recipe has them) come from default_rng([seed, 1 << 20])."""
    cfg = config(name)
    n_events = cfg["n_events"] if n_events is None else int(n_events)
    seed = cfg["seed"] if seed is None else int(seed)
    S = cfg["n_sectors"] if n_sectors is None else int(n_sectors)
    tracks = cfg["tracks"] if tracks is None else tracks
    noise = cfg["noise"] if noise is None else noise
    hidden = cfg["hidden"] if hidden is None else hidden
    misalign_sigma = cfg.get("misalign_sigma", 0.0) if misalign_sigma is None else misalign_sigma
    det = make_detector(S)
    params = make_compass_params(p_min_mev=cfg["p_min"],
                                 max_hits=cfg["max_hits"] if max_hits is None else max_hits,
                                 n_sectors_search=n_sectors_search)
    L, E = N_LAYERS, n_events
    delta_true = None
    if misalign_sigma and misalign_sigma > 0:
        delta_true = np.random.default_rng([seed, 1 << 20]).normal(
            0.0, misalign_sigma, L * S).astype(np.float32)

    def block(c):
        e0 = c * CHUNK_EVENTS
        return _chunk(np.random.default_rng([seed, c]), det, min(CHUNK_EVENTS, E - e0), S,
                      tracks, noise, hidden, delta_true, extra_padding_prob, with_truth,
                      outside_fraction)

    n_blocks = (E + CHUNK_EVENTS - 1) // CHUNK_EVENTS
    if n_blocks > 1:   # blocks are independent; numpy releases the GIL in the heavy steps
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1, n_blocks)) as pool:
            parts = list(pool.map(block, range(n_blocks)))
    else:
        parts = [block(c) for c in range(n_blocks)]

    def cat(key, dtype=None):
        if not parts:
            return np.zeros(0, dtype=dtype)
        return np.concatenate([p[key] for p in parts]).astype(dtype, copy=False) if dtype else \
            np.concatenate([p[key] for p in parts])

    words = cat("words", np.uint16)
    counts = cat("bank_counts", np.int64)
    bank_offsets = np.zeros(E * L * S + 1, dtype=np.uint32)
    np.cumsum(counts, out=bank_offsets[1:])
    n_velo = cat("n_velo", np.int64)
    velo_offsets = np.zeros(E + 1, dtype=np.uint32)
    np.cumsum(n_velo, out=velo_offsets[1:])
    batch = EventBatch(
        name=name, seed=seed, detector=det, params=params, n_events=E,
        words=words, bank_offsets=bank_offsets,
        velo_x=cat("vx", np.float32), velo_y=cat("vy", np.float32), velo_tx=cat("vtx", np.float32),
        velo_ty=cat("vty", np.float32), velo_offsets=velo_offsets,
        qop_true=cat("vqop", np.float64), n_layers_hit=cat("n_layers_hit", np.int8),
        delta_true=delta_true, outside=cat("outside", np.int8))
    if with_truth:
        tr = {}
        toff = 0
        tracks_ids = []
        for p in parts:
            t = p["truth"]["track"]
            tracks_ids.append(np.where(t >= 0, t + toff, t))
            toff += int(p["n_velo"].sum())
        tr["track"] = np.concatenate(tracks_ids).astype(np.int32) if parts else np.zeros(0, np.int32)
        for k in ("u_meas", "layer", "sector", "q", "size", "n_hidden", "n_noise"):
            tr[k] = np.concatenate([p["truth"][k] for p in parts]) if parts else np.zeros(0)
        batch.truth = tr
    return batch


def take_events(batch: EventBatch, events) -> EventBatch:
    """A new batch holding the given events (in the given order) of `batch`: their raw banks with
    rebased bank offsets and their VELO states.  Truth is not carried over."""
    ev = np.asarray(events, dtype=np.int64)
    L, S = N_LAYERS, batch.detector.n_sectors
    nb = L * S
    bo = batch.bank_offsets.astype(np.int64)
    vo = batch.velo_offsets.astype(np.int64)
    words, counts, tsel = [], [], []
    for e in ev:
        words.append(batch.words[bo[e * nb]:bo[(e + 1) * nb]])
        counts.append(np.diff(bo[e * nb:(e + 1) * nb + 1]))
        tsel.append(np.arange(vo[e], vo[e + 1]))
    tsel = np.concatenate(tsel) if tsel else np.zeros(0, np.int64)
    bank_offsets = np.zeros(ev.shape[0] * nb + 1, dtype=np.uint32)
    if counts:
        np.cumsum(np.concatenate(counts), out=bank_offsets[1:])
    velo_offsets = np.zeros(ev.shape[0] + 1, dtype=np.uint32)
    np.cumsum(vo[ev + 1] - vo[ev], out=velo_offsets[1:])
    return EventBatch(
        name=batch.name, seed=batch.seed, detector=batch.detector, params=batch.params,
        n_events=int(ev.shape[0]),
        words=np.concatenate(words) if words else np.zeros(0, np.uint16), bank_offsets=bank_offsets,
        velo_x=batch.velo_x[tsel], velo_y=batch.velo_y[tsel], velo_tx=batch.velo_tx[tsel],
        velo_ty=batch.velo_ty[tsel], velo_offsets=velo_offsets, qop_true=batch.qop_true[tsel],
        n_layers_hit=batch.n_layers_hit[tsel], delta_true=batch.delta_true,
        outside=batch.outside[tsel] if batch.outside is not None else None)
