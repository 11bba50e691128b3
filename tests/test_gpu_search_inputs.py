"""Compass on hit inputs the generator never produces, against the oracle, bit for bit.

The decoded hits of a seeded batch are altered before the search (the same arrays go to both sides):
per-hit strip y ranges (the per-hit y test), arbitrary positive weights including very large ones
(the rounding bound of the candidate pruning scales with them), a geometry with a non-positive kick
factor (pruning switched off) and VELO states with NaN.  Decoding itself is covered elsewhere.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu


def _search_both(b, det, d, vel=None):
    """Run the oracle and the GPU search on the same (possibly altered) hits and states."""
    vx, vy, vtx, vty = vel if vel is not None else (b.velo_x, b.velo_y, b.velo_tx, b.velo_ty)
    c = oracle.compass(det, b.params, b.n_events, d, vx, vy, vtx, vty, b.velo_offsets)
    geom = utc.Geometry(det, DEV)
    n = int(d["hit_offsets"][-1])
    hits = {"hit_offsets": torch.from_numpy(d["hit_offsets"].view(np.int32).copy()).to(DEV)}
    for k in ("u", "weight", "y_begin", "y_end"):
        hits[k] = torch.from_numpy(np.ascontiguousarray(d[k][:max(n, 1)], np.float32)).to(DEV)
    vdev = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV) for a in (vx, vy, vtx, vty)]
    vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(DEV)
    r = utc.compass_find(geom, b.params, b.n_events, hits, *vdev, vo)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in r.items()}
    assert np.array_equal(r["nhits"], c["nhits"]), np.nonzero(r["nhits"] != c["nhits"])[0][:10]
    assert np.array_equal(r["hit_idx"], c["hit_idx"])
    assert np.array_equal(r["qop"].view(np.uint32), c["qop"].view(np.uint32))
    assert np.array_equal(r["chi2"].view(np.uint32), c["chi2"].view(np.uint32))
    return r, c


@pytest.fixture(scope="module")
def base():
    b = synth.generate("batched", n_events=120, seed=71, with_truth=False)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    print(f"[search inputs] events={b.n_events} hits={int(d['hit_offsets'][-1])} tracks={b.n_tracks}",
          flush=True)
    return b, d


def test_per_hit_y_ranges(base):
    b, d = base
    rng = np.random.default_rng(5)
    n = int(d["hit_offsets"][-1])
    d2 = dict(d)
    d2["y_begin"] = rng.uniform(-700.0, 100.0, n).astype(np.float32)
    d2["y_end"] = (d2["y_begin"] + rng.uniform(0.0, 900.0, n)).astype(np.float32)
    r, c = _search_both(b, b.detector, d2)
    # the per-hit test must have removed some hits: fewer 4-hit tracks than with full-height strips
    assert (c["nhits"] == 4).sum() < (oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x,
                                                      b.velo_y, b.velo_tx, b.velo_ty,
                                                      b.velo_offsets)["nhits"] == 4).sum()


@pytest.mark.parametrize("scale", [1.0, 1e4])
def test_arbitrary_weights(base, scale):
    b, d = base
    rng = np.random.default_rng(6)
    n = int(d["hit_offsets"][-1])
    d2 = dict(d)
    d2["weight"] = (rng.uniform(1.0, 2000.0, n) * scale).astype(np.float32)
    r, c = _search_both(b, b.detector, d2)
    assert (c["nhits"] == 4).sum() > 0


def test_non_positive_kick_factor(base):
    b, d = base
    a = np.array(b.detector.a_kick, np.float32).copy()
    a[2] = -a[2]
    det = dataclasses.replace(b.detector, a_kick=a)
    r, c = _search_both(b, det, d)
    assert (c["nhits"] > 0).sum() > 0


def test_nan_states(base):
    b, d = base
    vx = b.velo_x.copy()
    vty = b.velo_ty.copy()
    vx[::7] = np.nan
    vty[3::11] = np.nan
    r, c = _search_both(b, b.detector, d, vel=(vx, b.velo_y, b.velo_tx, vty))
    assert (c["nhits"][::7] == 0).all()


def test_binding_rejects_wrong_tensors(base):
    """The library reads raw memory, so the binding refuses tensors of the wrong element type or
    layout instead of passing their pointers."""
    b = base[0]
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    vx64 = dv["vel"][0].double()
    with pytest.raises(ValueError):
        utc.compass_find(geom, b.params, b.n_events, hits, vx64, *dv["vel"][1:], dv["velo_offsets"])
    with pytest.raises(ValueError):
        utc.ut_decode(geom, dv["words"].float(), dv["bank_offsets"], b.n_events)
    strided = torch.stack([dv["words"], dv["words"]], dim=1)[:, 0]
    assert not strided.is_contiguous()
    with pytest.raises(ValueError):
        utc.ut_decode(geom, strided, dv["bank_offsets"], b.n_events)


def test_strip_ranges_with_nan_and_narrow_strips(base):
    """A strip range that is not a number makes its hit unusable; a few narrow strips in some
    events shrink the range that every strip of the event covers, so those events' tracks take the
    per-hit test while the other events' tracks skip it."""
    b, d = base
    rng = np.random.default_rng(9)
    n = int(d["hit_offsets"][-1])
    d2 = dict(d)
    yb = d["y_begin"][:n].copy()
    ye = d["y_end"][:n].copy()
    pick = rng.choice(n, 40, replace=False)
    yb[pick[:10]] = np.nan
    ye[pick[10:20]] = np.nan
    yb[pick[20:30]] = rng.uniform(-5.0, 5.0, 10).astype(np.float32)      # narrow strips
    ye[pick[30:40]] = rng.uniform(-5.0, 5.0, 10).astype(np.float32)
    d2["y_begin"], d2["y_end"] = yb, ye
    r, c = _search_both(b, b.detector, d2)
    assert (c["nhits"] > 0).sum() > 0
