"""GPU parity of the global event cut and of the track consolidation against their plain
definitions (oracle/select.py), and of the UT chain run on a cut batch."""
import numpy as np
import pytest
import torch

import oracle
import oracle.select as osel
import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def batch():
    b = synth.generate("realistic", n_events=300, seed=12, with_truth=False)
    per_event = np.diff(b.bank_offsets[::4 * b.detector.n_sectors].astype(np.int64))
    limit = int(np.median(per_event))
    print(f"[select] events={b.n_events} words={b.n_words} limit={limit}", flush=True)
    return b, to_dev(b), utc.Geometry(b.detector, DEV), limit


def _gpu_cut(b, dv, geom, limit):
    c = utc.ut_global_event_cut(geom, b.n_events, dv["words"], dv["bank_offsets"], *dv["vel"],
                                dv["velo_offsets"], limit)
    torch.cuda.synchronize()
    return c


@pytest.mark.parametrize("which", ["median", "none", "all"])
def test_event_cut_matches(batch, which):
    b, dv, geom, limit = batch
    lim = {"median": limit, "none": (1 << 32) - 1, "all": 0}[which]
    c = _gpu_cut(b, dv, geom, lim)
    o = osel.global_event_cut(b.detector.n_sectors, b.n_events, b.words, b.bank_offsets, b.velo_x,
                              b.velo_y, b.velo_tx, b.velo_ty, b.velo_offsets, lim)
    assert int(c["error_flags"].item()) == 0
    assert int(c["n_kept"].item()) == o["n_kept"]
    assert np.array_equal(c["keep"].cpu().numpy()[:b.n_events], o["keep"])
    assert np.array_equal(_u32(c["bank_offsets"]), o["bank_offsets"])
    assert np.array_equal(_u32(c["velo_offsets"]), o["velo_offsets"])
    nw, nt = o["words"].size, o["vx"].size
    assert np.array_equal(c["words"].cpu().numpy().view(np.uint16)[:nw], o["words"])
    for k in ("vx", "vy", "vtx", "vty"):
        assert np.array_equal(_u32(c[k])[:nt], o[k].view(np.uint32)), k


def test_chain_on_cut_batch(batch):
    """Decoding and tracking the cut batch equals the oracle on the oracle's cut batch."""
    b, dv, geom, limit = batch
    c = _gpu_cut(b, dv, geom, limit)
    hits = utc.ut_decode(geom, c["words"], c["bank_offsets"], b.n_events)
    res = utc.compass_find(geom, b.params, b.n_events, hits, c["vx"], c["vy"], c["vtx"], c["vty"],
                           c["velo_offsets"], n_tracks=b.n_tracks)
    torch.cuda.synchronize()
    o = osel.global_event_cut(b.detector.n_sectors, b.n_events, b.words, b.bank_offsets, b.velo_x,
                              b.velo_y, b.velo_tx, b.velo_ty, b.velo_offsets, limit)
    d = oracle.decode(b.detector, o["words"], o["bank_offsets"], b.n_events, hit_capacity=max(o["words"].size, 1))
    r = oracle.compass(b.detector, b.params, b.n_events, d, o["vx"], o["vy"], o["vtx"], o["vty"],
                       o["velo_offsets"])
    n = int(d["hit_offsets"][-1])
    assert np.array_equal(_u32(hits["hit_offsets"]), d["hit_offsets"])
    assert np.array_equal(_u32(hits["u"])[:n], d["u"][:n].view(np.uint32))
    nt = o["vx"].size
    assert np.array_equal(res["hit_idx"].cpu().numpy()[:nt], r["hit_idx"])
    assert np.array_equal(_u32(res["qop"])[:nt], r["qop"].view(np.uint32))


@pytest.mark.parametrize("name", ["realistic", "batched"])
def test_consolidate_matches(name):
    b = synth.generate(name, n_events=200, seed=21, with_truth=False)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    r = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    res = {k: torch.from_numpy(np.ascontiguousarray(r[k])).to(DEV) for k in ("nhits", "hit_idx", "qop", "chi2")}
    vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(DEV)
    g = utc.compass_consolidate(b.n_events, vo, res)
    torch.cuda.synchronize()
    o = osel.consolidate(b.n_events, b.velo_offsets, r["nhits"], r["hit_idx"], r["qop"], r["chi2"])
    nf = o["n_found"]
    assert int(g["n_found"].item()) == nf and nf > 0
    assert np.array_equal(_u32(g["offsets"]), o["offsets"])
    assert np.array_equal(g["velo"].cpu().numpy()[:nf], o["velo"])
    assert np.array_equal(g["hit_idx"].cpu().numpy()[:nf], o["hit_idx"])
    assert np.array_equal(g["nhits"].cpu().numpy()[:nf], o["nhits"])
    assert np.array_equal(_u32(g["qop"])[:nf], o["qop"].view(np.uint32))
    assert np.array_equal(_u32(g["chi2"])[:nf], o["chi2"].view(np.uint32))


def test_consolidate_empty():
    vo = torch.zeros(4, dtype=torch.int32, device=DEV)
    res = dict(nhits=torch.zeros(0, dtype=torch.int32, device=DEV),
               hit_idx=torch.zeros((0, 4), dtype=torch.int32, device=DEV),
               qop=torch.zeros(0, dtype=torch.float32, device=DEV),
               chi2=torch.zeros(0, dtype=torch.float32, device=DEV))
    g = utc.compass_consolidate(3, vo, res)
    torch.cuda.synchronize()
    assert int(g["n_found"].item()) == 0
    assert not g["offsets"].cpu().numpy().any()


def test_consolidate_unaligned_rows():
    """hit_idx rows that are not 16-byte aligned take the scalar copy; same result as aligned rows."""
    b = synth.generate("realistic", n_events=60, seed=23, with_truth=False)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    r = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    res = {k: torch.from_numpy(np.ascontiguousarray(r[k])).to(DEV) for k in ("nhits", "hit_idx", "qop", "chi2")}
    vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(DEV)
    n = b.n_tracks
    buf = torch.zeros(4 * n + 1, dtype=torch.int32, device=DEV)
    buf[1:] = res["hit_idx"].reshape(-1)
    shifted = dict(res, hit_idx=buf[1:].view(n, 4))
    assert shifted["hit_idx"].data_ptr() % 16 == 4
    g0 = utc.compass_consolidate(b.n_events, vo, res)
    g1 = utc.compass_consolidate(b.n_events, vo, shifted)
    torch.cuda.synchronize()
    nf = int(g0["n_found"].item())
    assert nf == int(g1["n_found"].item()) and nf > 0
    for k in ("offsets", "velo", "hit_idx", "nhits", "qop", "chi2"):
        a, e = g1[k], g0[k]
        if k != "offsets":
            a, e = a[:nf], e[:nf]
        assert torch.equal(a, e), k
