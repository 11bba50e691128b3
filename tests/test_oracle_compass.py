"""Pins of the oracle tracklet search (Section V) against brute force, closed forms and truth.

* windows: a linear scan over every hit of the allowed sectors (found through the LHCbID, not the
  offsets array) must give the same hit set, and a capped window must hold the hits nearest to the
  prediction;
* tracklets: every combination of one window hit or none per layer with at least three hits, assessed
  by the candidate predicate and the selection order, must give the oracle's choice;
* fit: hits placed exactly on the single-kick model give back the generated q/p, and the one-
  parameter weighted least squares agrees with numpy.linalg.lstsq;
* physics: most reconstructible synthetic tracks are found with their own hits.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests._truth import decoded_truth

f32 = np.float32
DIRS = ((0, 2, 1, 3), (3, 1, 2, 0))


def _run(b, **kw):
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                       b.velo_ty, b.velo_offsets, with_windows=True)
    return d, c


def _extrap(det, b, t):
    xs, yl, up = [], [], []
    for l in range(4):
        dz = f32(det.z_layer[l]) - f32(det.z_velo)
        x = f32(b.velo_x[t]) + f32(b.velo_tx[t]) * dz
        y = f32(b.velo_y[t]) + f32(b.velo_ty[t]) * dz
        xs.append(x); yl.append(y); up.append(x - y * f32(det.dxdy[l]))
    return xs, yl, up


def _event_of(b, t):
    return int(np.searchsorted(b.velo_offsets, t, side="right") - 1)


CASES = [
    dict(name="tiny", n_events=20, tracks=("fixed", 5)),
    dict(name="tiny", n_events=6, tracks=("fixed", 5), noise=("fixed", 20000), max_hits=4),
    dict(name="tiny", n_events=4, tracks=("fixed", 5), noise=("fixed", 20000), max_hits=8,
         n_sectors_search=1),
    dict(name="realistic", n_events=2, tracks=("fixed", 20), max_hits=3, n_sectors_search=3),
]


@pytest.mark.parametrize("case", CASES)
def test_windows_match_linear_scan(case):
    b = synth.generate(**case)
    det, par = b.detector, b.params
    d, c = _run(b)
    S = det.n_sectors
    n = int(d["hit_offsets"][-1])
    lid = d["lhcbid"][:n].astype(np.int64)
    hit_layer, hit_sector = lid >> 28, (lid >> 12) & 0xFFFF
    ho = d["hit_offsets"].astype(np.int64)
    W = f32(par.w0) + f32(par.kw) / f32(par.p_min)
    half = (par.n_sectors_search - 1) // 2
    checked_cap = 0
    for t in range(b.n_tracks):
        if not c["active"][t]:
            continue
        e = _event_of(b, t)
        xs, yl, up = _extrap(det, b, t)
        for l in range(4):
            cs = np.floor((up[l] - f32(det.u_min)) * f32(det.inv_sector_width))
            cc = int(min(max(cs, 0), S - 1))
            allowed = set(range(max(cc - half, 0), min(cc + half, S - 1) + 1))
            lo_ev, hi_ev = ho[(e * 4 + l) * S], ho[(e * 4 + l + 1) * S]
            cand = [i for i in range(lo_ev, hi_ev)
                    if hit_layer[i] == l and hit_sector[i] in allowed
                    and up[l] - W <= d["u"][i] <= up[l] + W]
            first, size = int(c["win_first"][t, l]), int(c["win_size"][t, l])
            got = list(range(first, first + size))
            if len(cand) <= par.max_hits:
                assert got == cand, (t, l)
            else:
                checked_cap += 1
                assert size == par.max_hits and set(got) <= set(cand)
                dist = {i: abs(f32(d["u"][i]) - up[l]) for i in cand}
                inside = max(dist[i] for i in got)
                outside = min(dist[i] for i in cand if i not in got)
                assert inside <= outside, (t, l)
    if case.get("max_hits", 8) <= 4:
        assert checked_cap > 0


def test_window_cap_tie_keeps_left():
    """Two hits at the same distance on either side: the right one is dropped."""
    det = synth.make_detector(32)
    par = synth.make_compass_params(max_hits=1, n_sectors_search=1)
    S = 32
    # one track along x = 10 mm with tx=ty=0 (so u = 10 at every layer), kick-free windows
    u_pred = f32(10.0)
    hits_u = [u_pred - f32(0.25), u_pred + f32(0.25)]
    ho = np.zeros(4 * S + 1, np.uint32)
    sector = int(np.floor((u_pred - f32(det.u_min)) * f32(det.inv_sector_width)))
    counts = np.zeros(4 * S, np.int64)
    for l in range(4):
        counts[l * S + sector] = 2
    ho[1:] = np.cumsum(counts)
    u = np.array(hits_u * 4, np.float32)
    hits = dict(hit_offsets=ho, u=u, weight=np.full(8, 400, np.float32),
                y_begin=np.full(8, -650, np.float32), y_end=np.full(8, 650, np.float32))
    c = oracle.compass(det, par, 1, hits, [10.0], [0.0], [0.0], [0.0],
                       np.array([0, 1], np.uint32), with_windows=True)
    assert list(c["win_first"][0]) == [0, 2, 4, 6]
    assert list(c["win_size"][0]) == [1, 1, 1, 1]


def _fit32(det, xs, yl, u, w, idx):
    Sar, Saa, r = f32(0), f32(0), {}
    for l in range(4):
        if idx[l] < 0:
            continue
        m = f32(u[idx[l]]) + yl[l] * f32(det.dxdy[l])
        r[l] = m - xs[l]
        wa = f32(w[idx[l]]) * f32(det.a_kick[l])
        Sar = Sar + wa * r[l]
        Saa = Saa + wa * f32(det.a_kick[l])
    q = Sar / Saa
    chi2 = f32(0)
    for l in range(4):
        if idx[l] < 0:
            continue
        e = r[l] - f32(det.a_kick[l]) * q
        chi2 = chi2 + (f32(w[idx[l]]) * e) * e
    return q, chi2


def _valid_in_dir(det, par, xs, yl, u, yb, ye, vtx, idx, dirn):
    A, B, C1, C2 = DIRS[dirn]
    if idx[A] < 0 or idx[B] < 0:
        return False
    for l in range(4):
        if idx[l] >= 0 and not (yb[idx[l]] <= yl[l] <= ye[idx[l]]):
            return False
    m = {l: f32(u[idx[l]]) + yl[l] * f32(det.dxdy[l]) for l in range(4) if idx[l] >= 0}
    inv = f32(1.0) / (f32(det.z_layer[B]) - f32(det.z_layer[A]))
    slope = (m[B] - m[A]) * inv
    if not (abs(slope - vtx) <= f32(par.slope_tol)):
        return False
    for Cl in (C1, C2):
        if idx[Cl] < 0:
            continue
        dd = f32(det.z_layer[Cl]) - f32(det.z_layer[A])
        xt = m[A] + slope * dd
        xv = m[A] + vtx * dd
        lo = min(xt, xv) - f32(par.completion_tol)
        hi = max(xt, xv) + f32(par.completion_tol)
        if not (lo <= m[Cl] <= hi):
            return False
    return True


@pytest.mark.parametrize("case", CASES)
def test_tracklets_match_brute_force(case):
    b = synth.generate(**case)
    det, par = b.detector, b.params
    d, c = _run(b)
    u, w, yb, ye = d["u"], d["weight"], d["y_begin"], d["y_end"]
    n_found = 0
    for t in range(b.n_tracks):
        if not c["active"][t]:
            assert c["nhits"][t] == 0
            continue
        xs, yl, _ = _extrap(det, b, t)
        vtx = f32(b.velo_tx[t])
        wins = [[-1] + list(range(int(c["win_first"][t, l]),
                                  int(c["win_first"][t, l] + c["win_size"][t, l])))
                for l in range(4)]
        best = None
        for dirn in (0, 1):
            for idx in itertools.product(*wins):
                nh = sum(i >= 0 for i in idx)
                if nh < 3 or not _valid_in_dir(det, par, xs, yl, u, yb, ye, vtx, idx, dirn):
                    continue
                q, chi2 = _fit32(det, xs, yl, u, w, idx)
                key = (-nh, float(chi2), tuple(idx))
                if best is None or key < best[0]:
                    best = (key, q, chi2, idx)
            if best is not None:
                break
        if best is None:
            assert c["nhits"][t] == 0 and list(c["hit_idx"][t]) == [-1] * 4
            continue
        n_found += 1
        assert list(c["hit_idx"][t]) == list(best[3]), t
        assert c["nhits"][t] == -best[0][0]
        assert c["qop"][t] == best[1] and c["chi2"][t] == best[2]
    assert n_found > 0


def test_duplicate_hits_tie_goes_to_lower_index():
    """Identical raw words give identical chi2; the lower hit index must win."""
    b = synth.generate("tiny", n_events=1, tracks=("fixed", 5))
    d0, c0 = _run(b)
    # duplicate the word of the layer-1 hit of every found track inside its bank
    words = list(b.words)
    off = b.bank_offsets.astype(np.int64).tolist()
    S = b.detector.n_sectors
    lid = d0["lhcbid"]
    dup_banks = set()
    for t in range(b.n_tracks):
        h = c0["hit_idx"][t, 1]
        if h >= 0:
            s = (int(lid[h]) >> 12) & 0xFFFF
            dup_banks.add((1 * S + s, int(lid[h])))
    new_words, new_off = [], [0]
    for bank in range(len(off) - 1):
        ws = words[off[bank]:off[bank + 1]]
        for (bb, idv) in dup_banks:
            if bb == bank:
                strip, frac = (idv >> 3) & 0x1FF, idv & 7
                ws = ws + [w for w in ws if (w >> 4) == ((strip << 3) | frac)][:1]
        new_words += ws
        new_off.append(len(new_words))
    b.words = np.array(new_words, np.uint16)
    b.bank_offsets = np.array(new_off, np.uint32)
    d, c = _run(b)
    for t in range(b.n_tracks):
        h = c["hit_idx"][t, 1]
        if h >= 0 and c0["hit_idx"][t, 1] >= 0:
            # the hit right after the chosen one is its duplicate
            assert d["lhcbid"][h] == d["lhcbid"][h + 1] and d["u"][h] == d["u"][h + 1]
            assert h == 0 or not (d["lhcbid"][h - 1] == d["lhcbid"][h] and
                                  d["weight"][h - 1] == d["weight"][h])


def _model_event(det, states, qops, y_extra=None):
    """Hit SoA of one event with one exact, unquantised model hit per track and layer."""
    S = det.n_sectors
    per_bank = {}
    for (x0, y0, tx, ty), q in zip(states, qops):
        for l in range(4):
            dz = float(det.z_layer[l]) - float(det.z_velo)
            x = x0 + tx * dz + q * float(det.a_kick[l])
            y = y0 + ty * dz
            u = x - y * float(det.dxdy[l])
            s = int(np.floor((u - det.u_min_f64) / 97.28))
            per_bank.setdefault(l * S + s, []).append(np.float32(u))
    ho = np.zeros(4 * S + 1, np.uint32)
    us = []
    for bank in range(4 * S):
        us += sorted(per_bank.get(bank, []))
        ho[bank + 1] = len(us)
    n = len(us)
    return dict(hit_offsets=ho, u=np.array(us, np.float32), weight=np.full(n, 400, np.float32),
                y_begin=np.full(n, -650, np.float32), y_end=np.full(n, 650, np.float32))


@pytest.mark.parametrize("spread", [(0.0, 1.0, 0.0005), (0.0, 300.0, 0.25)])
def test_closed_form_qop_recovery(spread):
    """Noise-free, unquantised hits on the single-kick model: the fit returns the generated q/p."""
    det = synth.make_detector(32)
    par = synth.make_compass_params()
    rng = np.random.default_rng(7)
    n = 40
    xy, ty_sp = spread[1], spread[2]
    x0 = rng.uniform(-xy, xy, n).astype(np.float32) * 0.01
    y0 = rng.uniform(-1, 1, n).astype(np.float32)
    tx = rng.uniform(-ty_sp, ty_sp, n).astype(np.float32)
    ty = rng.uniform(-ty_sp, ty_sp, n).astype(np.float32)
    q = (np.where(rng.random(n) < 0.5, -1, 1) / rng.uniform(3000, 20000, n))
    # one track per event so windows never mix tracks
    for t in range(n):
        st = [(float(x0[t]), float(y0[t]), float(tx[t]), float(ty[t]))]
        hits = _model_event(det, st, [q[t]])
        c = oracle.compass(det, par, 1, hits, x0[t:t + 1], y0[t:t + 1], tx[t:t + 1], ty[t:t + 1],
                           np.array([0, 1], np.uint32))
        assert c["nhits"][0] == 4
        # rounding bound: each residual carries a few float32 roundings of the magnitudes involved
        mags = []
        for l in range(4):
            dz = float(det.z_layer[l]) - float(det.z_velo)
            xs = abs(float(x0[t]) + float(tx[t]) * dz)
            yl = abs(float(y0[t]) + float(ty[t]) * dz) * abs(float(det.dxdy[l]))
            mags.append(xs + yl + float(np.abs(hits["u"]).max()) + 1.0)
        a = det.a_kick.astype(np.float64)
        bound = 6 * 2.0 ** -24 * max(mags) * a.sum() / (a * a).sum() + 1e-6 * abs(q[t])
        assert abs(float(c["qop"][0]) - q[t]) <= bound, (t, c["qop"][0], q[t], bound)
        assert float(c["chi2"][0]) <= 400 * 4 * (6 * 2.0 ** -24 * max(mags)) ** 2 * 16


def test_fit_matches_lstsq():
    """The 1-parameter weighted LSQ is lstsq on sqrt(w)-scaled rows (float64 reference)."""
    b = synth.generate("tiny", n_events=10)
    det = b.detector
    d, c = _run(b)
    checked = 0
    for t in range(b.n_tracks):
        if c["nhits"][t] < 3:
            continue
        rows, rhs, ws, aa, rr = [], [], [], [], []
        for l in range(4):
            h = c["hit_idx"][t, l]
            if h < 0:
                continue
            dz = float(det.z_layer[l]) - float(det.z_velo)
            xs = float(b.velo_x[t]) + float(b.velo_tx[t]) * dz
            yl = float(b.velo_y[t]) + float(b.velo_ty[t]) * dz
            r = float(d["u"][h]) + yl * float(det.dxdy[l]) - xs
            sw = np.sqrt(float(d["weight"][h]))
            rows.append([sw * float(det.a_kick[l])]); rhs.append(sw * r)
            ws.append(float(d["weight"][h])); aa.append(float(det.a_kick[l])); rr.append(r)
        q64 = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0][0]
        chi64 = sum(wi * (ri - ai * q64) ** 2 for wi, ai, ri in zip(ws, aa, rr))
        assert abs(float(c["qop"][t]) - q64) <= 2e-3 * abs(q64) + 2e-8
        assert abs(float(c["chi2"][t]) - chi64) <= 2e-3 * chi64 + 2e-3
        checked += 1
    assert checked > 400


def test_physics_efficiency_on_truth():
    """Reconstructible tracks (hits in >= 3 layers) are found with >= 70% of their own hits."""
    b = synth.generate("tiny")
    d, c = _run(b)
    hit_track, _, _ = decoded_truth(b)
    reco = b.n_layers_hit >= 3
    good = 0
    for t in np.nonzero(reco)[0]:
        idx = c["hit_idx"][t]
        nh = int(c["nhits"][t])
        if nh == 0:
            continue
        matched = sum(1 for h in idx if h >= 0 and hit_track[h] == t)
        good += matched >= 0.7 * nh
    eff = good / reco.sum()
    assert eff > 0.9, eff
    # the fitted q/p carries the charge for stiff-kick tracks
    found = c["nhits"] >= 3
    soft = found & (np.abs(b.qop_true) > 2e-4)
    agree = np.mean(np.sign(c["qop"][soft]) == np.sign(b.qop_true[soft]))
    assert agree > 0.95, agree


def test_out_of_acceptance_tracks_are_skipped():
    b = synth.generate("tiny", n_events=2)
    b.velo_ty = b.velo_ty.copy()
    b.velo_ty[:10] = 0.6          # y at the last layer far above the 650 mm planes
    b.velo_x = b.velo_x.copy()
    b.velo_x[10:20] = 3000.0      # beyond the last sector
    d, c = _run(b)
    assert not c["active"][:20].any() and c["active"][20:].all()
    assert np.all(c["nhits"][:20] == 0) and np.all(c["hit_idx"][:20] == -1)


def test_layer_overflow_flag():
    """An (event, layer) with more than 32767 hits cannot be addressed by 16-bit windows."""
    det = synth.make_detector(32)
    par = synth.make_compass_params()
    S = 32
    ho = np.zeros(2 * 4 * S + 1, np.uint32)
    counts = np.zeros(2 * 4 * S, np.int64)
    counts[0] = 40000                       # event 0, layer 0, sector 0
    ho[1:] = np.cumsum(counts)
    n = int(ho[-1])
    hits = dict(hit_offsets=ho, u=np.full(n, -1556.0, np.float32), weight=np.full(n, 400, np.float32),
                y_begin=np.full(n, -650, np.float32), y_end=np.full(n, 650, np.float32))
    c = oracle.compass(det, par, 2, hits, [0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0],
                       np.array([0, 1, 2], np.uint32), with_windows=True)
    assert c["flags"] & oracle.FLAG_LAYER_OVERFLOW
    assert c["active"][0] == 0 and c["active"][1] == 1


def test_greedy_variant_properties():
    """The paper's variant: with a budget of one tracklet the result is the first tracklet in window
    order; a budget larger than the number of pairs gives the minimum over one candidate per pair,
    which can never beat the exhaustive minimum."""
    b = synth.generate("tiny", n_events=6, seed=13)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    ex = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                        b.velo_offsets)
    big = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=b.params.max_hits,
                                    n_sectors_search=b.params.n_sectors_search, max_tracklets=1 << 20)
    one = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=b.params.max_hits,
                                    n_sectors_search=b.params.n_sectors_search, max_tracklets=1)
    g = oracle.compass(b.detector, big, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    g1 = oracle.compass(b.detector, one, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                        b.velo_offsets)
    # the same tracks get a tracklet (one exists iff some passing pair has a compatible hit)
    assert np.array_equal(g["nhits"] > 0, ex["nhits"] > 0)
    assert np.array_equal(g1["nhits"] > 0, ex["nhits"] > 0)
    both = (ex["nhits"] == 4) & (g["nhits"] == 4)
    assert both.sum() > 0
    # the exhaustive minimum is never worse; where the greedy choice is a 4-hit one it is one of
    # the exhaustive candidates, so its chi2 is at least the exhaustive 4-hit minimum
    assert np.all(ex["chi2"][both] <= g["chi2"][both])
    assert np.all(ex["nhits"] >= g["nhits"])
    # a budget of one tracklet can never select better than a larger budget
    sel = (g1["nhits"] == g["nhits"]) & (g["nhits"] > 0)
    assert np.all(g["chi2"][sel] <= g1["chi2"][sel])
    assert np.all(np.isfinite(g["chi2"][g["nhits"] > 0]))


def test_greedy_variant_equals_exhaustive_for_single_hit_windows():
    """With one hit per window every pair has at most one compatible hit per completion layer, so
    the closest-hit choice and the exhaustive minimum coincide (budget above the pair count)."""
    b = synth.generate("realistic", n_events=8, seed=14)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    kw = dict(p_min_mev=float(b.params.p_min), max_hits=1, n_sectors_search=5)
    ex = oracle.compass(b.detector, synth.make_compass_params(**kw), b.n_events, d, b.velo_x, b.velo_y,
                        b.velo_tx, b.velo_ty, b.velo_offsets)
    g = oracle.compass(b.detector, synth.make_compass_params(**kw, max_tracklets=1000), b.n_events, d,
                       b.velo_x, b.velo_y, b.velo_tx, b.velo_ty, b.velo_offsets)
    assert (ex["nhits"] == 4).sum() > 0
    for k in ("nhits", "hit_idx", "qop", "chi2"):
        assert np.array_equal(ex[k], g[k]), k
