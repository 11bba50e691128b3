"""GPU Compass on the hand-worked fixtures of tests/golden/ and on tracks outside the planes, against
the expected labels and the oracle, bit for bit (Sections V-A and V-B).

The fixtures decide the walk order of the paper's search (central sector first), the A-major pair
order, the closest completion hit, the weight and NaN rules of the selection and the acceptance
boundary at the first and the last layer; the generated batches put a fifth of the VELO tracks
outside the planes in each of the four ways the generator knows.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2002_11529_amd as utc
from tests.golden_search import N_SECTORS, build_event, load_acceptance_tracks, load_search_cases
from tests.gpu_helpers import DEV, assert_compass_equal, oracle_windows_rel, to_dev

pytestmark = pytest.mark.gpu

CASES = load_search_cases()


def _hits_dev(hits):
    n = max(int(hits["hit_offsets"][-1]), 1)
    out = {"hit_offsets": torch.from_numpy(hits["hit_offsets"].view(np.int32).copy()).to(DEV)}
    for k in ("u", "weight", "y_begin", "y_end"):
        a = np.zeros(n, np.float32)
        a[:hits[k].shape[0]] = hits[k]
        out[k] = torch.from_numpy(a).to(DEV)
    return out


def _find(det, par, n_events, hits, states, velo_offsets):
    geom = utc.Geometry(det, DEV)
    vdev = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV) for a in states]
    vo = torch.from_numpy(np.asarray(velo_offsets, np.uint32).view(np.int32).copy()).to(DEV)
    r = utc.compass_find(geom, par, n_events, _hits_dev(hits), *vdev, vo, windows=True)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in r.items()}
    r["error_flags"] = int(r["error_flags"].view(np.uint32)[0])
    return r


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_search_fixture_on_gpu(case):
    print(f"[golden] {case['name']} params={case['params']}", flush=True)
    det, par, hits, st, expect = build_event(case)
    vo = np.array([0, 1], np.uint32)
    r = _find(det, par, 1, hits, st, vo)
    c = oracle.compass(det, par, 1, hits, *st, vo)
    assert r["error_flags"] == 0
    assert list(r["hit_idx"][0]) == expect
    assert_compass_equal(r, c)


def test_acceptance_fixture_on_gpu():
    states, active = load_acceptance_tracks()
    det = synth.make_detector(N_SECTORS)
    par = synth.make_compass_params()
    hits = dict(hit_offsets=np.zeros(4 * N_SECTORS + 1, np.uint32), u=np.zeros(1, np.float32),
                weight=np.zeros(1, np.float32), y_begin=np.zeros(1, np.float32),
                y_end=np.zeros(1, np.float32))
    n = len(active)
    r = _find(det, par, 1, hits, [states[:, k] for k in range(4)], np.array([0, n], np.uint32))
    # a searched track gets a window (first hit 0, size 0 here); a filtered one the marker -1
    assert list((r["windows"][:, 0, 0] >= 0).astype(np.uint8)) == list(active)
    assert (r["nhits"] == 0).all()


@pytest.fixture(scope="module", params=["realistic", "batched"])
def outside_batch(request):
    n = {"realistic": 150, "batched": 150}[request.param]
    b = synth.generate(request.param, n_events=n, seed=83, with_truth=False, outside_fraction=0.2)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    print(f"[outside {request.param}] events={b.n_events} tracks={b.n_tracks}", flush=True)
    return b, d


def test_tracks_outside_the_planes(outside_batch):
    b, d = outside_batch
    codes = b.outside
    # every way of leaving the planes is present, each on at least 3 % of the tracks
    for k in (synth.events.OUTSIDE_Y_LAST, synth.events.OUTSIDE_Y_FIRST, synth.events.OUTSIDE_U_LAST,
              synth.events.OUTSIDE_U_FIRST):
        assert (codes == k).mean() > 0.03, k
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    res = utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"],
                           windows=True)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in res.items()}
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets, with_windows=True)
    assert_compass_equal(r, c, b, d)
    out = codes != synth.events.OUTSIDE_NONE
    assert not c["active"][out].any()
    assert (r["windows"][out][:, :, 0] == -1).all() and (r["nhits"][out] == 0).all()
    assert c["active"][~out].mean() > 0.99


@pytest.fixture(scope="module")
def wide_batch():
    b = synth.generate("realistic", n_events=60, seed=89, with_truth=False)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    print(f"[wide windows] events={b.n_events} tracks={b.n_tracks}", flush=True)
    return b, d


@pytest.mark.parametrize("max_hits,budget", [(8, 1), (8, 2), (8, 5), (16, 3), (32, 7), (16, 0)])
def test_wide_windows_walk_order(wide_batch, max_hits, budget):
    """Windows of +-40 mm straddle sector edges often, so the walk order of the paper's search
    (central sector first) decides which tracklets a binding budget keeps."""
    b, d = wide_batch
    p = synth.make_compass_params(max_hits=max_hits, n_sectors_search=5, max_tracklets=budget,
                                  w0_mm=39.0)
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    hits = {k: torch.from_numpy(np.ascontiguousarray(d[k]).view(
        np.int32 if d[k].dtype == np.uint32 else d[k].dtype)).to(DEV)
        for k in ("hit_offsets", "u", "weight", "y_begin", "y_end")}
    res = utc.compass_find(geom, p, b.n_events, hits, *dv["vel"], dv["velo_offsets"], windows=True)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in res.items()}
    c = oracle.compass(b.detector, p, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets, with_windows=True)
    assert_compass_equal(r, c, b, d)
    assert (c["nhits"] > 0).mean() > 0.5
