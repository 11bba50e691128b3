"""The physics-efficiency figures (synth/efficiency.py) on the oracle's tracks: the decoded-hit
truth map, sane values, and the trend of the paper's efficiency table (more hit candidates per
window: higher efficiency, flattening)."""
import numpy as np

import oracle
import synth
from synth.efficiency import decoded_hit_truth, efficiency


def _run(b, **params):
    p = synth.make_compass_params(p_min_mev=1500.0, **params)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    c = oracle.compass(b.detector, p, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    return d, c


def test_decoded_hit_truth_matches_positions():
    b = synth.generate("tiny", n_events=5, seed=2)
    d, _ = _run(b, max_hits=8, n_sectors_search=5)
    tr = decoded_hit_truth(b)
    n = int(d["hit_offsets"][-1])
    assert tr.size == n
    # the map agrees with the decoded hits: a VELO particle's hit lies within one fine bin (1/8
    # strip) of the position the generator measured for it
    valid = (b.words & 0xF) != 0
    bank = np.repeat(np.arange(b.bank_offsets.size - 1), np.diff(b.bank_offsets.astype(np.int64)))
    idx = np.nonzero(valid)[0]
    order = np.lexsort((idx, b.words[idx], bank[idx]))
    um = b.truth["u_meas"][idx[order]]
    sel = tr >= 0
    assert sel.sum() > 0
    assert np.all(np.abs(d["u"][:n][sel] - um[sel]) <= b.detector.pitch8 * 0.5 + 1e-3)


def test_efficiency_values_and_trend():
    b = synth.generate("realistic", n_events=30, seed=9)
    effs = {}
    for m in (1, 2, 4, 8):
        _, c = _run(b, max_hits=m, n_sectors_search=5)
        effs[m] = efficiency(b, c["hit_idx"], c["nhits"])
    e8 = effs[8]
    assert e8["efficiency"] > 0.85 and e8["clone_rate"] < 0.01 and e8["fake_rate"] < 0.15
    # a second candidate per window helps a lot, beyond four the gain is gone (flattening)
    assert effs[2]["efficiency"] > effs[1]["efficiency"] + 0.05
    assert abs(effs[8]["efficiency"] - effs[4]["efficiency"]) < effs[2]["efficiency"] - effs[1]["efficiency"]
    assert effs[1]["fake_rate"] > effs[8]["fake_rate"]
    # one sector can only lose the tracks whose window crosses a sector edge
    _, c1 = _run(b, max_hits=8, n_sectors_search=1)
    assert efficiency(b, c1["hit_idx"], c1["nhits"])["efficiency"] <= e8["efficiency"]


def test_association_threshold_is_exact():
    """Section III-B: a track reconstructs a particle when 70 % of its hits belong to it.  7 of 10
    is exactly 70 % (a floating-point 0.7 * 10 would exceed 7); 3 of 4 and 4 of 4 pass, 2 of 3 does
    not; noise (-1) and hidden particles (-2) are never associated."""
    from synth.efficiency import associated
    assert associated(np.array([5] * 7 + [1, 2, 3])) == 5
    assert associated(np.array([5] * 6 + [1, 2, 3, 4])) == -1
    assert associated(np.array([4, 4, 4, -1])) == 4
    assert associated(np.array([4, 4, 9])) == -1
    assert associated(np.array([-1, -1, -1])) == -1
    assert associated(np.array([-2, -2, -2, 3])) == -1


def test_clone_and_fake_rates_on_a_hand_built_event():
    """One event, four VELO particles P0..P3 and noise, hits placed by hand (one word per hit, words
    in ascending value inside each bank, so the decoded order is the listed order):
      P0, P1: a hit in every layer (reconstructible); P2: layers 0, 1, 2 (reconstructible);
      P3: layers 0, 1 only (not reconstructible); one noise hit in layer 3.
    Found tracks: VELO slot 0 = P0's four hits (reconstructs P0); slot 1 = P0's hits in layers 0-2
    plus the noise hit (3 of 4 = 75 %: a clone of P0); slot 2 = P2's hits in layers 0 and 1 plus P1's
    layer-2 hit (2 of 3 = 67 %: a fake); slot 3 found nothing.
    Hence efficiency = 1 of 3 reconstructible particles, clone rate = 1 of 3 found tracks, fake
    rate = 1 of 3 found tracks."""
    from synth.events import EventBatch
    from synth.efficiency import efficiency
    S = 2
    det = synth.make_detector(S)
    # (layer, particle) in the order of the hits inside bank (layer, sector 0)
    layout = {0: [0, 1, 2, 3], 1: [0, 1, 2, 3], 2: [0, 1, 2], 3: [0, 1, -1]}
    words, truth, bank_offsets, index = [], [], [0], {}
    for l in range(4):
        for s in range(S):
            if s == 0:
                for k, pid in enumerate(layout[l]):
                    index[(l, pid)] = len(words)
                    words.append(((10 + k) << 7) | (0 << 4) | 1)   # strip 10+k, size 1
                    truth.append(pid)
            bank_offsets.append(len(words))
    n_layers_hit = np.array([4, 4, 3, 2], np.int8)
    z = np.zeros(4, np.float32)
    b = EventBatch(name="hand", seed=0, detector=det, params=synth.make_compass_params(),
                   n_events=1, words=np.array(words, np.uint16),
                   bank_offsets=np.array(bank_offsets, np.uint32), velo_x=z, velo_y=z, velo_tx=z,
                   velo_ty=z, velo_offsets=np.array([0, 4], np.uint32), qop_true=np.zeros(4),
                   n_layers_hit=n_layers_hit, truth={"track": np.array(truth, np.int32)})
    hit_idx = np.full((4, 4), -1, np.int32)
    hit_idx[0] = [index[(l, 0)] for l in range(4)]
    hit_idx[1] = [index[(0, 0)], index[(1, 0)], index[(2, 0)], index[(3, -1)]]
    hit_idx[2] = [index[(0, 2)], index[(1, 2)], index[(2, 1)], -1]
    nhits = np.array([4, 4, 3, 0], np.int32)
    e = efficiency(b, hit_idx, nhits)
    assert e["reconstructible"] == 3 and e["found"] == 3
    assert e["efficiency"] == 1 / 3
    assert e["clone_rate"] == 1 / 3
    assert e["fake_rate"] == 1 / 3
