"""Pins of the event cut and consolidation definitions (oracle/select.py)."""
import numpy as np

import oracle
import oracle.select as osel
import synth


def _cut(b, max_words):
    return osel.global_event_cut(b.detector.n_sectors, b.n_events, b.words, b.bank_offsets, b.velo_x,
                                 b.velo_y, b.velo_tx, b.velo_ty, b.velo_offsets, max_words)


def test_cut_without_limit_is_identity():
    b = synth.generate("tiny", n_events=7, seed=3)
    c = _cut(b, 1 << 30)
    assert c["n_kept"] == 7
    assert np.array_equal(c["words"], b.words) and np.array_equal(c["bank_offsets"], b.bank_offsets)
    assert np.array_equal(c["velo_offsets"], b.velo_offsets) and np.array_equal(c["vtx"], b.velo_tx)


def test_cut_at_zero_empties_every_event():
    b = synth.generate("tiny", n_events=5, seed=3)
    c = _cut(b, 0)
    assert c["n_kept"] == 0 and c["words"].size == 0 and c["vx"].size == 0
    assert not c["bank_offsets"].any() and not c["velo_offsets"].any()


def test_cut_keeps_the_small_events_and_their_decoding():
    b = synth.generate("batched", n_events=40, seed=8)
    per_event = np.diff(b.bank_offsets[::4 * b.detector.n_sectors].astype(np.int64))
    limit = int(np.median(per_event))
    c = _cut(b, limit)
    kept = np.nonzero(per_event <= limit)[0]
    assert c["n_kept"] == kept.size and np.array_equal(np.nonzero(c["keep"])[0], kept)
    # decoding the cut batch gives, for the kept events, exactly the decoding of those events alone
    d_cut = oracle.decode(b.detector, c["words"], c["bank_offsets"], b.n_events)
    sub = synth.take_events(b, kept)
    d_sub = oracle.decode(sub.detector, sub.words, sub.bank_offsets, sub.n_events)
    n = int(d_sub["hit_offsets"][-1])
    assert int(d_cut["hit_offsets"][-1]) == n
    for k in ("lhcbid", "u", "weight"):
        assert np.array_equal(d_cut[k][:n], d_sub[k][:n])
    assert np.array_equal(c["velo_offsets"][kept + 1] - c["velo_offsets"][kept],
                          np.diff(b.velo_offsets.astype(np.int64))[kept])


def test_consolidate_maps_back_and_counts():
    rng = np.random.default_rng(4)
    n_events, vo = 6, np.array([0, 3, 3, 10, 11, 20, 25], np.uint32)
    n = int(vo[-1])
    nhits = rng.choice([0, 3, 4], n).astype(np.int32)
    hit_idx = rng.integers(-1, 1000, (n, 4)).astype(np.int32)
    qop = rng.normal(size=n).astype(np.float32)
    chi2 = rng.random(n).astype(np.float32)
    c = osel.consolidate(n_events, vo, nhits, hit_idx, qop, chi2)
    assert c["n_found"] == int((nhits > 0).sum())
    assert np.all(np.diff(c["velo"]) > 0)
    assert np.array_equal(c["hit_idx"], hit_idx[c["velo"]]) and np.array_equal(c["qop"], qop[c["velo"]])
    ev = np.repeat(np.arange(n_events), np.diff(vo.astype(np.int64)))
    assert np.array_equal(np.diff(c["offsets"].astype(np.int64)), np.bincount(ev[nhits > 0], minlength=n_events))
