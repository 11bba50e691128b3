"""GPU parity: the HIP path through the C ABI against the oracle, element by element.

Decoded hits, hit offsets, windows and selected hit indices are compared bit for bit; q/p and chi2
too, since both sides evaluate the same float32 operation sequence (the tolerance the workload
definition allows, 1e-5 relative, is therefore not needed).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import (DEV, gpu_run, oracle_run, assert_decode_equal, assert_compass_equal,
                               to_dev)

pytestmark = pytest.mark.gpu

CASES = {
    "tiny": dict(name="tiny"),
    "tiny_padding": dict(name="tiny", n_events=37, extra_padding_prob=0.1, seed=11),
    "realistic_100": dict(name="realistic", n_events=100),
    "batched_300": dict(name="batched", n_events=300),
    "pileup_20": dict(name="pileup", n_events=20),
    "dense_cap4": dict(name="tiny", n_events=12, noise=("fixed", 20000), max_hits=4),
    "one_sector": dict(name="tiny", n_events=12, noise=("fixed", 8000), n_sectors_search=1),
    "three_sectors": dict(name="realistic", n_events=10, n_sectors_search=3, max_hits=16),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    b = synth.generate(**CASES[request.param], with_truth=False)
    print(f"[case {request.param}] events={b.n_events} words={b.n_words} tracks={b.n_tracks}",
          flush=True)
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    return b, h, r, d, c


def test_decode_bit_exact(case):
    b, h, r, d, c = case
    assert h["error_flags"] == 0 and d["flags"] == 0
    assert_decode_equal(h, d)


def test_compass_bit_exact(case):
    b, h, r, d, c = case
    assert r["error_flags"] == 0 and c["flags"] == 0
    assert_compass_equal(r, c, b, d)
    assert (c["nhits"] > 0).sum() > 0


def test_full_realistic_workload():
    """The full 1000-event, 200-sector workload in the default launch shape, every output."""
    b = synth.generate("realistic", with_truth=False)
    print(f"[realistic full] words={b.n_words} tracks={b.n_tracks}", flush=True)
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)


def test_pileup_sampled_events():
    """High-occupancy events (up to ~3000 tracks, 16-hit windows): 200 events, every output."""
    b = synth.generate("pileup", n_events=200, seed=55, with_truth=False)
    print(f"[pileup 200] words={b.n_words} tracks={b.n_tracks}", flush=True)
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)


@pytest.mark.parametrize("launch", [dict(block=64), dict(block=128, grid=7), dict(block=512, grid=3)])
def test_decode_launch_shapes_agree(launch):
    b = synth.generate("batched", n_events=60, with_truth=False)
    h0, r0, *_ = gpu_run(b)
    h1, r1, *_ = gpu_run(b, launch_decode=launch,
                         launch_find=dict(block=min(launch["block"], 256), grid=launch.get("grid", 0)))
    n = int(h0["hit_offsets"][-1])
    assert np.array_equal(h0["hit_offsets"], h1["hit_offsets"])
    for k in ("lhcbid", "u", "weight"):
        assert np.array_equal(h0[k][:n], h1[k][:n])
    for k in ("hit_idx", "nhits", "qop", "chi2", "windows"):
        assert np.array_equal(r0[k], r1[k])


def test_repeat_runs_identical():
    b = synth.generate("realistic", n_events=50, with_truth=False)
    h0, r0, *_ = gpu_run(b)
    h1, r1, *_ = gpu_run(b)
    n = int(h0["hit_offsets"][-1])
    for k in ("lhcbid", "u", "weight"):
        assert h0[k][:n].tobytes() == h1[k][:n].tobytes()
    for k in ("hit_idx", "nhits", "qop", "chi2"):
        assert r0[k].tobytes() == r1[k].tobytes()


def test_empty_and_ragged_events():
    """Events without tracks, without hits, and a mix of sizes."""
    b = synth.generate("tiny", n_events=9, tracks=("fixed", 3))
    # drop all tracks of events 2 and 5, and all hits of events 3 and 5
    vo = b.velo_offsets.astype(np.int64)
    keep = np.ones(b.n_tracks, bool)
    for e in (2, 5):
        keep[vo[e]:vo[e + 1]] = False
    counts = np.diff(vo)
    counts[[2, 5]] = 0
    b.velo_offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    for a in ("velo_x", "velo_y", "velo_tx", "velo_ty"):
        setattr(b, a, getattr(b, a)[keep])
    S = b.detector.n_sectors
    off = b.bank_offsets.astype(np.int64)
    wkeep = np.ones(b.n_words, bool)
    for e in (3, 5):
        wkeep[off[e * 4 * S]:off[(e + 1) * 4 * S]] = False
    nb = np.diff(off)
    for e in (3, 5):
        nb[e * 4 * S:(e + 1) * 4 * S] = 0
    b.words = b.words[wkeep]
    b.bank_offsets = np.concatenate([[0], np.cumsum(nb)]).astype(np.uint32)
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)


def test_single_event_and_zero_events():
    b = synth.generate("tiny", n_events=1)
    h, r, *_ = gpu_run(b)
    d, c = oracle_run(b)
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)
    import paper_2002_11529_amd as utc
    geom = utc.Geometry(b.detector, DEV)
    hits = utc.ut_decode(geom, torch.zeros(0, dtype=torch.int16, device=DEV),
                         torch.zeros(1, dtype=torch.int32, device=DEV), 0, hit_capacity=0)
    torch.cuda.synchronize()
    assert int(hits["hit_offsets"][0]) == 0


def test_bad_bank_order_and_capacity_flags():
    b = synth.generate("tiny", n_events=4)
    off = b.bank_offsets.copy()
    k = 40
    while off[k + 1] == off[k]:
        k += 1
    off[k + 1] = off[k] - 1
    b.bank_offsets = off
    d, c = oracle_run(b)
    h, r, *_ = gpu_run(b)
    assert d["flags"] & oracle.FLAG_BANK_ORDER and h["error_flags"] & oracle.FLAG_BANK_ORDER
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)
    b2 = synth.generate("tiny", n_events=4)
    cap = b2.n_valid_words - 17
    # compass_find needs every hit the offsets refer to, so only the decoder runs here
    d2, _ = oracle_run(b2, hit_capacity=cap, find=False)
    h2, _, *_ = gpu_run(b2, hit_capacity=cap, find=False)
    assert d2["flags"] & oracle.FLAG_CAPACITY and h2["error_flags"] & oracle.FLAG_CAPACITY
    assert np.array_equal(h2["hit_offsets"], d2["hit_offsets"])
    assert np.array_equal(h2["u"][:cap], d2["u"][:cap])


def test_oversized_bank_flagged():
    b = synth.generate("tiny", n_events=2)
    S = b.detector.n_sectors
    # append 9000 padding+valid words to bank 5 of event 1
    bank = 4 * S + 5
    off = b.bank_offsets.astype(np.int64)
    extra = np.full(9000, (3 << 7) | 1, np.uint16)
    words = np.concatenate([b.words[:off[bank + 1]], extra, b.words[off[bank + 1]:]])
    off2 = off.copy()
    off2[bank + 1:] += 9000
    b.words, b.bank_offsets = words, off2.astype(np.uint32)
    d, c = oracle_run(b)
    h, r, *_ = gpu_run(b)
    assert d["flags"] & oracle.FLAG_BANK_SIZE and h["error_flags"] & oracle.FLAG_BANK_SIZE
    assert_decode_equal(h, d)
    assert_compass_equal(r, c, b, d)
