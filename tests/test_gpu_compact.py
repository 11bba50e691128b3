"""GPU parity of the compact hit form: the decoder run without the per-hit layer constants (z,
y_begin, y_end) writes the same remaining arrays, and the search run without the per-hit y ranges
(each strip then spans the detector's y range) gives the same tracks, bit for bit, as the full
form and the oracle."""
import numpy as np
import pytest
import torch

import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev, oracle_run, assert_compass_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["realistic", "batched", "pileup"])
def batch(request):
    n = {"realistic": 150, "batched": 60, "pileup": 10}[request.param]
    b = synth.generate(request.param, n_events=n, seed=73, with_truth=False)
    print(f"[compact {request.param}] events={b.n_events} tracks={b.n_tracks} words={b.n_words}",
          flush=True)
    return b, to_dev(b), utc.Geometry(b.detector, DEV)


def _np(res):
    r = {k: v.cpu().numpy() for k, v in res.items()}
    r["error_flags"] = int(r["error_flags"].view(np.uint32)[0])
    return r


def test_compact_decode_matches_full(batch):
    b, dv, geom = batch
    full = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    comp = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, compact=True)
    torch.cuda.synchronize()
    assert not any(k in comp for k in ("z", "y_begin", "y_end"))
    assert int(comp["error_flags"].item()) == 0
    n = int(full["hit_offsets"][-1].item())
    assert n > 0
    assert torch.equal(comp["hit_offsets"], full["hit_offsets"])
    for k in ("lhcbid", "u", "weight"):
        a = comp[k][:n].cpu().numpy().view(np.uint32)
        e = full[k][:n].cpu().numpy().view(np.uint32)
        assert np.array_equal(a, e), k


def test_compact_search_matches_full_and_oracle(batch):
    b, dv, geom = batch
    full = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    comp = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, compact=True)
    rf = _np(utc.compass_find(geom, b.params, b.n_events, full, *dv["vel"], dv["velo_offsets"]))
    rc = _np(utc.compass_find(geom, b.params, b.n_events, comp, *dv["vel"], dv["velo_offsets"]))
    torch.cuda.synchronize()
    d, c = oracle_run(b)
    assert rc["error_flags"] == 0
    assert_compass_equal(rc, c)
    assert_compass_equal(rf, c)
    assert (c["nhits"] > 0).sum() > 0


def test_search_rejects_half_y_range(batch):
    """Only one of the two per-hit y arrays is a caller error, caught before any launch."""
    b, dv, geom = batch
    full = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    torch.cuda.synchronize()
    half = {k: v for k, v in full.items() if k != "y_end"}
    with pytest.raises(RuntimeError):
        utc.compass_find(geom, b.params, b.n_events, half, *dv["vel"], dv["velo_offsets"])
