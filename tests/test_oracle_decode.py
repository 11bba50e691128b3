"""Pins of the oracle decoder against what the generator and the hit definition fix.

Section IV: each raw bank is decoded into hits carrying a 32-bit LHCbID, z, x at y=0, yBegin, yEnd
and a weight, stored as a structure of arrays with an offsets array per sector group, hits ordered
inside each group.  The pins below do not re-run the decoder's arithmetic: they compare its output
with the generator's own record of what it encoded.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._truth import decoded_word_index, word_bank_ids

PITCH = 0.19


def _decode(b):
    return oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)


@pytest.mark.parametrize("name,n_events", [("tiny", 100), ("realistic", 20)])
def test_round_trip_per_bank(name, n_events):
    """Multiset of (layer, sector, strip, fraction, size) per bank equals what was encoded."""
    b = synth.generate(name, n_events=n_events, extra_padding_prob=0.02)
    d = _decode(b)
    assert d["flags"] == 0
    S = b.detector.n_sectors
    tr = b.truth
    valid = tr["size"] > 0
    bank = word_bank_ids(b.bank_offsets)
    enc = np.stack([bank[valid], tr["layer"][valid], tr["sector"][valid], tr["q"][valid],
                    tr["size"][valid]], axis=1).astype(np.int64)
    ho = d["hit_offsets"].astype(np.int64)
    n = int(ho[-1])
    assert n == valid.sum()
    hit_bank = np.repeat(np.arange(ho.shape[0] - 1), np.diff(ho))
    lid = d["lhcbid"][:n].astype(np.int64)
    size_of_weight = {float(b.detector.weight_by_size[k]): k for k in (1, 2, 3)}
    size = np.array([size_of_weight[float(w)] for w in d["weight"][:n]])
    dec = np.stack([hit_bank, lid >> 28, (lid >> 12) & 0xFFFF, lid & 0xFFF, size], axis=1)
    # the bank index also fixes (event, layer, sector): check the LHCbID agrees with it
    assert np.array_equal(dec[:, 1], (hit_bank // S) % 4)
    assert np.array_equal(dec[:, 2], hit_bank % S)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert np.array_equal(key(enc), key(dec))


def test_counts_and_offsets():
    b = synth.generate("tiny", n_events=30, extra_padding_prob=0.05)
    d = _decode(b)
    ho = d["hit_offsets"].astype(np.int64)
    off = b.bank_offsets.astype(np.int64)
    valid = (b.words & 0xF) != 0
    cs = np.concatenate([[0], np.cumsum(valid.astype(np.int64))])
    per_bank = cs[off[1:]] - cs[off[:-1]]
    assert ho[0] == 0
    assert np.array_equal(np.diff(ho), per_bank)


def test_u_matches_generated_position():
    """x at y=0 lies within half a 1/8-strip bin of the smeared position the generator encoded."""
    b = synth.generate("tiny")
    d = _decode(b)
    wi = decoded_word_index(b.words, b.bank_offsets)
    umeas = b.truth["u_meas"][wi]
    track_hit = np.isfinite(umeas)
    assert track_hit.sum() > 15000
    u = d["u"][:wi.shape[0]].astype(np.float64)
    err = np.abs(u - umeas)[track_hit]
    ulp = np.spacing(np.abs(u[track_hit]).astype(np.float32)).astype(np.float64)
    assert np.all(err <= PITCH / 16 + ulp)
    # and it is not trivially small: the quantisation is visible
    assert err.max() > PITCH / 32


def test_hits_sorted_by_x_within_layer():
    b = synth.generate("realistic", n_events=10)
    d = _decode(b)
    ho = d["hit_offsets"].astype(np.int64)
    S = b.detector.n_sectors
    for e in range(b.n_events):
        for l in range(4):
            lo, hi = ho[(e * 4 + l) * S], ho[(e * 4 + l + 1) * S]
            u = d["u"][lo:hi]
            assert np.all(np.diff(u) >= 0)


def test_constant_fields():
    b = synth.generate("tiny", n_events=5)
    d = _decode(b)
    n = int(d["hit_offsets"][-1])
    layer = d["lhcbid"][:n] >> 28
    assert np.array_equal(d["z"][:n], b.detector.z_layer[layer])
    assert np.all(d["y_begin"][:n] == -650.0) and np.all(d["y_end"][:n] == 650.0)
    assert set(np.unique(d["weight"][:n])) <= set(b.detector.weight_by_size[1:4].tolist())


def test_hand_decoded_words():
    """A hand-worked example: the words of tests/golden/decode_words.txt and their fields."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "decode_words.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    det = synth.make_detector(32)
    S = 32
    by_bank = {}
    for r in rows:
        by_bank.setdefault(int(r[0]) * S + int(r[1]), []).append(r)
    banks = np.zeros(4 * S + 1, np.uint32)
    words, expected = [], []
    for bnk in range(4 * S):
        rs = by_bank.get(bnk, [])
        words += [int(r[2], 16) for r in reversed(rs)]      # shuffled order in the raw bank
        expected += rs
        banks[bnk + 1] = len(words)
    d = oracle.decode(det, np.array(words, np.uint16), banks, 1)
    assert int(d["hit_offsets"][-1]) == len(rows)
    for k, r in enumerate(expected):
        assert d["lhcbid"][k] == int(r[3], 16)
        u = np.float32(d["u"][k])
        assert abs(float(u) - float(r[4])) <= float(np.spacing(abs(u)))
        assert float(d["weight"][k]) == pytest.approx(float(r[5]), rel=1e-6)
        assert float(d["z"][k]) == float(det.z_layer[int(r[0])])


def test_bad_bank_order_flagged():
    b = synth.generate("tiny", n_events=3)
    off = b.bank_offsets.copy()
    k = 7
    while off[k + 1] == off[k]:
        k += 1
    off[k + 1] = off[k] - 1 if off[k] > 0 else 0
    if off[k + 1] >= off[k]:
        pytest.skip("no bank to corrupt")
    d = oracle.decode(b.detector, b.words, off, b.n_events)
    assert d["flags"] & oracle.FLAG_BANK_ORDER
    assert d["hit_offsets"][k + 1] == d["hit_offsets"][k]


def test_capacity_flagged_without_overrun():
    b = synth.generate("tiny", n_events=3)
    n = b.n_valid_words
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events, hit_capacity=n - 10)
    assert d["flags"] & oracle.FLAG_CAPACITY
    assert d["hit_offsets"][-1] == n
    full = _decode(b)
    assert np.array_equal(d["u"], full["u"][:n - 10])


@pytest.mark.parametrize("name,n_events", [("tiny", 20), ("realistic", 3), ("pileup", 1)])
def test_u_is_one_correctly_rounded_fma(name, n_events):
    """u = fma(8*strip + fraction, pitch/8, u0) rounded once (Section IV, x at y = 0).  In binary64
    the product and the sum are exact here: q < 2^12, pitch8 and u0 are binary32 values with
    24-bit significands, the product's exponent range is small and every term is a multiple of
    2^-30 below 2^14, so the exact value fits the 53-bit significand.  One rounding of that binary64
    value to binary32 is therefore the correctly rounded fused result, bit for bit; a decoder that
    rounds the product before the sum differs on some hits."""
    b = synth.generate(name, n_events=n_events)
    d = _decode(b)
    det = b.detector
    S = det.n_sectors
    n = int(d["hit_offsets"][-1])
    lid = d["lhcbid"][:n].astype(np.int64)
    layer, sector = lid >> 28, (lid >> 12) & 0xFFFF
    q = ((lid >> 3) & 0x1FF) * 8 + (lid & 7)
    p8 = np.float64(np.float32(det.pitch8))
    u0 = np.asarray(det.u0, np.float32).astype(np.float64)[layer * S + sector]
    exact = q.astype(np.float64) * p8 + u0
    # the binary64 sum is exact: subtracting the terms back leaves no remainder
    assert np.array_equal(exact - u0, q.astype(np.float64) * p8)
    assert np.array_equal(d["u"][:n].view(np.uint32), exact.astype(np.float32).view(np.uint32))
    two_roundings = (np.float32(q.astype(np.float32) * np.float32(det.pitch8)) +
                     np.asarray(det.u0, np.float32)[layer * S + sector])
    assert (two_roundings != d["u"][:n]).any()
