"""GPU parity of the paper's search variant (closest completion hit per layer, first N tracklets,
Section V-B) against the oracle, bit for bit, for several tracklet budgets and workloads."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev, assert_compass_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["realistic", "batched", "pileup"])
def decoded(request):
    n = {"realistic": 120, "batched": 80, "pileup": 12}[request.param]
    b = synth.generate(request.param, n_events=n, seed=61, with_truth=False)
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    print(f"[variant {request.param}] events={b.n_events} tracks={b.n_tracks}", flush=True)
    return b, dv, geom, hits, d


@pytest.mark.parametrize("budget", [1, 2, 4, 16, 100000])
def test_variant_matches_oracle(decoded, budget):
    b, dv, geom, hits, d = decoded
    p = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=b.params.max_hits,
                                  n_sectors_search=b.params.n_sectors_search, max_tracklets=budget)
    res = utc.compass_find(geom, p, b.n_events, hits, *dv["vel"], dv["velo_offsets"])
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in res.items()}
    r["error_flags"] = int(r["error_flags"].view(np.uint32)[0])
    c = oracle.compass(b.detector, p, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    assert r["error_flags"] == 0
    assert_compass_equal(r, c)
    assert (c["nhits"] > 0).sum() > 0


@pytest.mark.parametrize("m,budget", [(1, 0), (2, 0), (4, 0), (1, 1), (2, 2), (4, 4), (16, 16)])
def test_sweep_configurations(decoded, m, budget):
    """The configurations of the efficiency sweep (windows of m hits; the exhaustive search, or the
    paper's search with a budget of m tracklets) on every workload."""
    b, dv, geom, hits, d = decoded
    p = synth.make_compass_params(p_min_mev=float(b.params.p_min), max_hits=m,
                                  n_sectors_search=b.params.n_sectors_search, max_tracklets=budget)
    res = utc.compass_find(geom, p, b.n_events, hits, *dv["vel"], dv["velo_offsets"])
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in res.items()}
    c = oracle.compass(b.detector, p, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    assert_compass_equal(r, c)
    assert (c["nhits"] > 0).sum() > 0
