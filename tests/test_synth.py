"""Synthetic event generator: determinism, recipe shapes and raw-bank format."""
import numpy as np
import pytest

import synth


def test_seeded_determinism():
    a = synth.generate("tiny", n_events=10)
    b = synth.generate("tiny", n_events=10)
    assert np.array_equal(a.words, b.words)
    assert np.array_equal(a.bank_offsets, b.bank_offsets)
    assert np.array_equal(a.velo_tx, b.velo_tx)
    c = synth.generate("tiny", n_events=10, seed=99)
    assert not np.array_equal(a.words, c.words)


def test_tiny_shape():
    b = synth.generate("tiny")
    det = b.detector
    assert b.n_events == 100 and det.n_sectors == 32
    assert b.n_tracks == 5000
    assert np.all(np.diff(b.velo_offsets.astype(np.int64)) == 50)
    # 50 tracks * 4 layers * 0.97 + 200 noise hits per event
    per_event = b.n_valid_words / b.n_events
    assert 380 < per_event < 410
    assert b.bank_offsets.shape[0] == 100 * 4 * 32 + 1


def test_realistic_shape():
    b = synth.generate("realistic", n_events=50)
    per_event = b.n_valid_words / b.n_events
    assert 2800 < per_event < 3200          # ~3000 UT hits per event
    noise = np.count_nonzero(b.truth["track"] == synth.events.TRUTH_NOISE) / b.n_events
    assert 0.2 < noise / per_event < 0.3    # 25% noise


def test_batched_uneven_sizes():
    b = synth.generate("batched", n_events=300, with_truth=False)
    nt = np.diff(b.velo_offsets.astype(np.int64))
    assert nt.min() >= 10 and nt.max() <= 1500
    assert 150 < np.median(nt) < 260
    ratio = (b.n_valid_words - 500 * b.n_events) / nt.sum()
    assert 13.5 < ratio < 16.5              # ~15 hits per VELO track


def test_raw_bank_format():
    b = synth.generate("tiny", n_events=20, extra_padding_prob=0.05)
    off = b.bank_offsets.astype(np.int64)
    assert off[0] == 0 and off[-1] == b.n_words and np.all(np.diff(off) >= 0)
    # every bank has an even number of words (32-bit aligned)
    assert np.all(np.diff(off) % 2 == 0)
    w = b.words.astype(np.int64)
    size = w & 0xF
    tr = b.truth
    assert np.array_equal(size, tr["size"])
    pad = size == 0
    assert np.all(tr["track"][pad] == synth.events.TRUTH_PADDING)
    assert np.all(w[pad] == 0)
    q = ((w >> 7) << 3) | ((w >> 4) & 7)
    assert np.array_equal(q[~pad], tr["q"][~pad])
    assert set(np.unique(size[~pad])) <= {1, 2, 3}


def test_detector_description():
    det = synth.make_detector(32)
    assert det.u0.dtype == np.float32 and det.u0.shape == (128,)
    # sectors tile the layer side by side; bin 0 centre sits pitch/16 right of the sector edge
    assert abs(float(det.u0[0]) - (-16 * 97.28 + 0.19 / 16)) < 1e-3
    assert abs(float(det.u0[31]) - (15 * 97.28 + 0.19 / 16)) < 1e-3
    assert det.dxdy[0] == 0 and det.dxdy[3] == 0 and det.dxdy[1] == -det.dxdy[2] > 0
    # single kick: deflection at mid-UT (z = 2490 mm) equals K * qop
    assert abs(0.5 * (float(det.a_kick[1]) + float(det.a_kick[2])) - 1200.0) < 1e-3
    with pytest.raises(ValueError):
        synth.make_detector(31)


def test_take_events_matches_slices():
    import oracle
    b = synth.generate("tiny", n_events=6, seed=9)
    sub = synth.take_events(b, [4, 1])
    S = b.detector.n_sectors
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    ds = oracle.decode(sub.detector, sub.words, sub.bank_offsets, sub.n_events)
    for k, e in enumerate((4, 1)):
        ho = d["hit_offsets"].astype(np.int64)
        a0, a1 = ho[e * 4 * S], ho[(e + 1) * 4 * S]
        s0 = ds["hit_offsets"][k * 4 * S]
        assert np.array_equal(ds["hit_offsets"][k * 4 * S:(k + 1) * 4 * S + 1] - s0,
                              (ho[e * 4 * S:(e + 1) * 4 * S + 1] - a0).astype(np.uint32))
        assert np.array_equal(ds["u"][s0:s0 + a1 - a0], d["u"][a0:a1])
        t0, t1 = b.velo_offsets[e], b.velo_offsets[e + 1]
        u0, u1 = sub.velo_offsets[k], sub.velo_offsets[k + 1]
        assert np.array_equal(sub.velo_tx[u0:u1], b.velo_tx[t0:t1])


def test_outside_fraction_places_tracks_outside_the_planes():
    """The generator's outside_fraction option moves VELO states so that their straight line leaves
    the planes at exactly one of the two checked layers; the oracle filters them out (Section V-A)
    and keeps every other track.  Without the option the batch is unchanged."""
    import oracle
    from synth.events import OUTSIDE_NONE
    b0 = synth.generate("realistic", n_events=30, with_truth=False)
    b = synth.generate("realistic", n_events=30, with_truth=False, outside_fraction=0.4)
    assert np.array_equal(b0.words, synth.generate("realistic", n_events=30, with_truth=False).words)
    assert (b0.outside == OUTSIDE_NONE).all()
    codes = np.bincount(b.outside, minlength=5)
    assert codes[1:].min() > 0.05 * b.n_tracks      # every way is well represented
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                       b.velo_ty, b.velo_offsets, with_windows=True)
    assert np.array_equal(c["active"] == 0, b.outside != OUTSIDE_NONE)
    # the moved tracks still leave hits in the layers they cross inside the planes
    assert (b.n_layers_hit[b.outside != OUTSIDE_NONE] >= 3).mean() > 0.2
