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
