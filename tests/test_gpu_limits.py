"""GPU parity at the limits of the interface: the largest window (UTC_MAX_WINDOW_HITS slots), the
largest geometry (8192 sectors per layer), a bank of exactly UTC_MAX_BANK_WORDS words, and an
(event, layer) with more hits than 16-bit windows can address.  Every case is compared with the
oracle element by element (decoded hits, offsets, windows, selected hits, q/p, chi2, flags)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import gpu_run, oracle_run, assert_decode_equal, assert_compass_equal

pytestmark = pytest.mark.gpu

MAX_WINDOW_HITS = 32
MAX_BANK_WORDS = 8192
MAX_SECTORS = 8192


def _check(b, flags=0):
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    # the search raises its flags in the decoder's flag word
    assert d["flags"] == flags & ~oracle.FLAG_LAYER_OVERFLOW
    assert r["error_flags"] == (d["flags"] | c["flags"]) == flags
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)
    return d, c


def test_full_32_hit_windows():
    """Dense events and a low momentum cut: most windows hold the full 32 slots, so every bit of
    the 32-bit slot masks is in use."""
    b = synth.generate("tiny", n_events=6, seed=31, noise=("fixed", 20000), with_truth=False)
    b.params = synth.make_compass_params(p_min_mev=150.0, max_hits=MAX_WINDOW_HITS, n_sectors_search=5)
    print(f"[limits max window] events={b.n_events} tracks={b.n_tracks}", flush=True)
    d, c = _check(b)
    assert (c["win_size"] == MAX_WINDOW_HITS).mean() > 0.5
    assert (c["nhits"] > 0).mean() > 0.9


@pytest.mark.parametrize("max_hits", [8, MAX_WINDOW_HITS])
def test_largest_geometry(max_hits):
    """8192 sectors per layer: the bank offsets of an event fill most of the LDS, the decoder and
    the search shrink their workgroups to fit."""
    b = synth.generate("tiny", n_events=3, seed=32, n_sectors=MAX_SECTORS, with_truth=False)
    b.params = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=max_hits,
                                         n_sectors_search=5)
    print(f"[limits S={MAX_SECTORS} M={max_hits}] events={b.n_events} tracks={b.n_tracks}", flush=True)
    d, c = _check(b)
    assert (c["nhits"] > 0).mean() > 0.9


def test_bank_of_the_largest_size():
    """A bank of exactly UTC_MAX_BANK_WORDS words is decoded (ranked against the whole bank a chunk
    at a time through LDS), not flagged."""
    b = synth.generate("tiny", n_events=2, seed=33, with_truth=False)
    S = b.detector.n_sectors
    bank = (1 * 4 + 2) * S + 7          # event 1, layer 2, sector 7
    off = b.bank_offsets.astype(np.int64)
    have = int(off[bank + 1] - off[bank])
    rng = np.random.default_rng(5)
    n = MAX_BANK_WORDS - have
    strip = rng.integers(0, 512, n)
    frac = rng.integers(0, 8, n)
    size = np.where(rng.random(n) < 0.1, 0, rng.integers(1, 16, n))   # 10 % padding
    extra = ((strip << 7) | (frac << 4) | size).astype(np.uint16)
    b.words = np.concatenate([b.words[:off[bank + 1]], extra, b.words[off[bank + 1]:]])
    off[bank + 1:] += n
    b.bank_offsets = off.astype(np.uint32)
    assert int(off[bank + 1] - off[bank]) == MAX_BANK_WORDS
    print(f"[limits bank] words={b.n_words}", flush=True)
    _check(b)


@pytest.mark.parametrize("n_extra,tile", [(1500, 0), (700, 4), (3000, 6)])
def test_banks_larger_than_the_lds_chunk(n_extra, tile):
    """Banks with more words than the decoder's LDS chunk (about 900 words at the default tile, a
    few hundred at small tiles) are ranked a chunk at a time through LDS; several such banks in one
    unit, duplicated words (ties keep bank order), padding in between."""
    b = synth.generate("tiny", n_events=3, seed=35, with_truth=False)
    S = b.detector.n_sectors
    rng = np.random.default_rng(n_extra)
    for bank in ((2 * 4 + 1) * S + 12, (2 * 4 + 1) * S + 17, (0 * 4 + 3) * S + 3):
        off = b.bank_offsets.astype(np.int64)
        strip = rng.integers(0, 64, n_extra)          # few distinct positions: many equal words
        frac = rng.integers(0, 8, n_extra)
        size = np.where(rng.random(n_extra) < 0.1, 0, rng.integers(1, 4, n_extra))
        extra = ((strip << 7) | (frac << 4) | size).astype(np.uint16)
        b.words = np.concatenate([b.words[:off[bank + 1]], extra, b.words[off[bank + 1]:]])
        off[bank + 1:] += n_extra
        b.bank_offsets = off.astype(np.uint32)
    print(f"[limits large banks] extra={n_extra} tile={tile} words={b.n_words}", flush=True)
    h, r, *_ = gpu_run(b, launch_decode=dict(block=256, grid=0, tile=tile), find=False)
    d, c = oracle_run(b, find=False)
    assert d["flags"] == 0 and h["error_flags"] == 0
    assert_decode_equal(h, d)


def _insert_words(b, bank, extra):
    """Append the words `extra` to bank `bank` of batch b (offsets of the later banks shifted)."""
    off = b.bank_offsets.astype(np.int64)
    b.words = np.concatenate([b.words[:off[bank + 1]], np.asarray(extra, np.uint16), b.words[off[bank + 1]:]])
    off[bank + 1:] += len(extra)
    b.bank_offsets = off.astype(np.uint32)


@pytest.mark.parametrize("tile", [0, 4])
def test_crowded_sort_bins(tile):
    """Banks that fit the decoder's LDS chunk but crowd its sort bins (each bank is cut into as
    many bins of the word's strip and fraction as it has hits): every word of a bank equal, all
    hits on two strips, hits only at both ends of the strip range (the first and the last bin),
    a one-hit bank and a bank of padding words only, in the units of two events; at the default
    tile the units are staged whole, at 4 KiB they are cut into chunks between banks."""
    b = synth.generate("tiny", n_events=3, seed=36, with_truth=False)
    S = b.detector.n_sectors
    rng = np.random.default_rng(36)
    w = lambda strip, frac, size: ((np.asarray(strip) << 7) | (np.asarray(frac) << 4) | np.asarray(size))
    n = 160
    cases = {
        (0 * 4 + 1) * S + 3: np.full(n, w(200, 5, 3)),                                   # all equal
        (0 * 4 + 1) * S + 4: w(rng.choice([17, 18], n), rng.integers(0, 8, n), rng.integers(1, 16, n)),
        (0 * 4 + 1) * S + 9: w(rng.choice([0, 511], n), rng.choice([0, 7], n), rng.integers(1, 3, n)),
        (0 * 4 + 1) * S + 10: w([300], [2], [4]),                                          # one hit
        (0 * 4 + 1) * S + 11: w(rng.integers(0, 512, 40), rng.integers(0, 8, 40), 0),     # padding only
        (2 * 4 + 3) * S + 0: w(rng.integers(250, 254, n), rng.integers(0, 8, n),
                               np.where(rng.random(n) < 0.2, 0, rng.integers(1, 16, n))),
        (2 * 4 + 3) * S + 31: np.full(n, w(511, 7, 15)),                                  # the last bin
    }
    # insert from the last bank backwards so that the earlier offsets stay valid
    for bank in sorted(cases, reverse=True):
        _insert_words(b, bank, cases[bank].astype(np.uint16))
    print(f"[limits crowded bins] tile={tile} words={b.n_words}", flush=True)
    h, r, *_ = gpu_run(b, launch_decode=dict(block=256, grid=0, tile=tile), find=False)
    d, c = oracle_run(b, find=False)
    assert d["flags"] == 0 and h["error_flags"] == 0
    assert_decode_equal(h, d)


def test_layer_beyond_16_bit_windows():
    """Event 0, layer 0 holds 40000 hits (five banks of 8000): the search flags the overflow and
    gives that event's tracks no candidates; the other event is searched as usual."""
    b = synth.generate("tiny", n_events=2, seed=34, with_truth=False)
    S = b.detector.n_sectors
    off = b.bank_offsets.astype(np.int64)
    rng = np.random.default_rng(6)
    parts, last = [], 0
    new_off = off.copy()
    added = 0
    for bank in range(5):              # event 0, layer 0, sectors 0..4
        parts.append(b.words[last:off[bank + 1]])
        n = 8000 - int(off[bank + 1] - off[bank])
        strip = rng.integers(0, 512, n)
        frac = rng.integers(0, 8, n)
        parts.append(((strip << 7) | (frac << 4) | 1).astype(np.uint16))
        added += n
        new_off[bank + 1] += added
        last = int(off[bank + 1])
    parts.append(b.words[last:])
    new_off[6:] = off[6:] + added
    b.words = np.concatenate(parts)
    b.bank_offsets = new_off.astype(np.uint32)
    print(f"[limits layer overflow] words={b.n_words}", flush=True)
    d, c = _check(b, flags=oracle.FLAG_LAYER_OVERFLOW)
    t0 = int(b.velo_offsets[1])
    assert not c["active"][:t0].any() and (c["nhits"][t0:] > 0).mean() > 0.9


def test_fit_gradient_on_the_largest_geometry():
    """8192 sectors per layer: the 4S offset sums no longer fit in LDS and are accumulated in place
    in the workspace; per-track terms bit for bit, sums within one ulp of the oracle's."""
    import torch
    import paper_2002_11529_amd as utc
    from tests.gpu_helpers import DEV
    b = synth.generate("tiny", n_events=20, seed=35, n_sectors=MAX_SECTORS, with_truth=False)
    h, r, geom, hits, res, dv = gpu_run(b)
    d, c = oracle_run(b)
    keep = c["nhits"] >= 3
    print(f"[limits fitgrad S={MAX_SECTORS}] tracks={int(keep.sum())}", flush=True)
    kd = torch.from_numpy(keep).to(DEV)
    rng = np.random.default_rng(7)
    q = (c["qop"][keep].astype(np.float64) * (1 + rng.normal(0, 0.05, int(keep.sum())))).astype(np.float32)
    off = rng.normal(0, 0.05, 4 * MAX_SECTORS).astype(np.float32)
    g = utc.compass_fit_grad(geom, res["hit_idx"][kd].contiguous(), hits["u"], hits["weight"], hits["lhcbid"],
                             *[v[kd].contiguous() for v in dv["vel"]], torch.from_numpy(q).to(DEV),
                             torch.from_numpy(off).to(DEV), grad_scale=0.5)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = oracle.fit_grad(b.detector, c["hit_idx"][keep], d["u"], d["weight"], d["lhcbid"], b.velo_x[keep],
                        b.velo_y[keep], b.velo_tx[keep], b.velo_ty[keep], q, off, grad_scale=0.5,
                        precision="f32")
    assert np.array_equal(g["chi2_track"].view(np.uint32), o["chi2_track"].view(np.uint32))
    assert np.array_equal(g["grad_qop"].view(np.uint32), o["grad_qop"].view(np.uint32))
    go, oo = g["grad_offsets"].astype(np.float64), o["grad_offsets"]
    assert np.all(np.abs(go - oo) <= np.spacing(np.abs(oo)))
    assert np.count_nonzero(oo) > 20
    assert g["chi2_total"][0] == pytest.approx(o["chi2_total"], rel=1e-12)


@pytest.mark.parametrize("n_search", [15, 65])
def test_wide_sector_search(n_search):
    """Searches over 15 sectors, and over more sectors than a layer has (the range is clamped)."""
    b = synth.generate("tiny", n_events=10, seed=36, noise=("fixed", 3000), with_truth=False)
    b.params = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=b.params.max_hits,
                                         n_sectors_search=n_search)
    print(f"[limits sectors searched {n_search}] tracks={b.n_tracks}", flush=True)
    d, c = _check(b)
    assert (c["nhits"] > 0).mean() > 0.9


def test_words_not_16_byte_aligned():
    """A word buffer that starts 2 bytes past a 16-byte boundary takes the decoder's scalar loads;
    the result is the same as from an aligned buffer (and the oracle's)."""
    import torch
    import paper_2002_11529_amd as utc
    from tests.gpu_helpers import DEV, to_dev
    b = synth.generate("realistic", n_events=40, seed=37, with_truth=False)
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    padded = torch.zeros(b.n_words + 1, dtype=torch.int16, device=DEV)
    padded[1:] = dv["words"]
    shifted = padded[1:]
    assert shifted.data_ptr() % 16 == 2
    ref = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    out = utc.ut_decode(geom, shifted, dv["bank_offsets"], b.n_events)
    torch.cuda.synchronize()
    n = int(ref["hit_offsets"][-1])
    assert torch.equal(ref["hit_offsets"], out["hit_offsets"])
    for k in ("lhcbid", "z", "u", "y_begin", "y_end", "weight"):
        assert torch.equal(ref[k][:n], out[k][:n]), k
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    assert np.array_equal(out["u"][:n].cpu().numpy().view(np.uint32), d["u"][:n].view(np.uint32))
