"""Parity at the workloads' full sizes, in the autotuned launch shapes that the benchmark times.

* realistic: 1000 events (200 sectors): every decoded hit and every track against the oracle.
* batched: 20000 uneven events (32 sectors): every decoded hit and every track against the oracle.
* pileup: 10000 high-occupancy events (200 sectors, 16-hit windows): every decoded hit, every track
  and the fraction of VELO tracks with a candidate against the oracle, run on event slices over the
  host's CPUs.
* fitgrad: 21000 events, about 1.05 million frozen tracks: chi2 and gradients of all of them against
  the float32 oracle and the binary64 reference.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu

L = 4


def _run_tuned(b):
    dv = to_dev(b)
    geom = utc.Geometry(b.detector, DEV)
    t = utc.autotune(geom, b.params, b.n_events, dv["words"], dv["bank_offsets"], *dv["vel"],
                     dv["velo_offsets"], reps=5)
    print(f"[{b.name} full] events={b.n_events} words={b.n_words} tracks={b.n_tracks} "
          f"launch decode={t['decode']} find={t['find']}", flush=True)
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, launch=t["decode"])
    res = utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"],
                           launch=t["find"])
    torch.cuda.synchronize()
    return geom, dv, hits, res


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _common_properties(b, hits, res):
    """Checks over every event: flags clear, hit count = valid words, selected hits inside the
    track's own event and in distinct layers."""
    assert int(hits["error_flags"].item()) == 0 and int(res["error_flags"].item()) == 0
    ho = _u32(hits["hit_offsets"]).astype(np.int64)
    assert np.all(np.diff(ho) >= 0)
    assert ho[-1] == b.n_valid_words
    S = b.detector.n_sectors
    nh = res["nhits"].cpu().numpy()
    idx = res["hit_idx"].cpu().numpy().astype(np.int64)
    assert set(np.unique(nh).tolist()) <= {0, 3, 4}
    assert np.array_equal((idx >= 0).sum(axis=1), nh)
    ev = np.repeat(np.arange(b.n_events), np.diff(b.velo_offsets.astype(np.int64)))
    for l in range(L):
        lo = ho[(ev * L + l) * S]
        hi = ho[(ev * L + l + 1) * S]
        sel = idx[:, l] >= 0
        assert np.all((idx[sel, l] >= lo[sel]) & (idx[sel, l] < hi[sel])), l
    return nh


def test_realistic_full_every_output():
    b = synth.generate("realistic", with_truth=False)
    geom, dv, hits, res = _run_tuned(b)
    _common_properties(b, hits, res)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx, b.velo_ty,
                       b.velo_offsets)
    n = int(d["hit_offsets"][-1])
    assert np.array_equal(_u32(hits["hit_offsets"]), d["hit_offsets"])
    for k in ("lhcbid", "u", "weight", "z", "y_begin", "y_end"):
        assert np.array_equal(_u32(hits[k])[:n], d[k][:n].view(np.uint32)), k
    assert np.array_equal(res["hit_idx"].cpu().numpy(), c["hit_idx"])
    assert np.array_equal(res["nhits"].cpu().numpy(), c["nhits"])
    for k in ("qop", "chi2"):
        assert np.array_equal(_u32(res[k]), c[k].view(np.uint32)), k


def test_batched_full_every_output():
    b = synth.generate("batched", with_truth=False)
    geom, dv, hits, res = _run_tuned(b)
    _common_properties(b, hits, res)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events, hit_capacity=b.n_words)
    n = int(d["hit_offsets"][-1])
    assert np.array_equal(_u32(hits["hit_offsets"]), d["hit_offsets"])
    for k in ("lhcbid", "z", "u", "y_begin", "y_end", "weight"):
        assert np.array_equal(_u32(hits[k][:n]), d[k][:n].view(np.uint32)), k
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                       b.velo_ty, b.velo_offsets)
    assert np.array_equal(res["nhits"].cpu().numpy(), c["nhits"])
    assert np.array_equal(res["hit_idx"].cpu().numpy(), c["hit_idx"])
    assert np.array_equal(_u32(res["qop"]), c["qop"].view(np.uint32))
    assert np.array_equal(_u32(res["chi2"]), c["chi2"].view(np.uint32))


def _oracle_slices(b, threads):
    """The oracle on contiguous event slices of `b`, one thread per slice (events are independent;
    the oracle's C calls release the interpreter lock).  Returns [(first event, end event, decoded
    hits, tracks)] with hit offsets and indices local to the slice."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = max(1, min(threads, len(os.sched_getaffinity(0)), b.n_events))
    cuts = np.linspace(0, b.n_events, n + 1).astype(np.int64)

    def run(k):
        sub = synth.take_events(b, np.arange(cuts[k], cuts[k + 1]))
        d = oracle.decode(sub.detector, sub.words, sub.bank_offsets, sub.n_events,
                          hit_capacity=sub.n_words)
        c = oracle.compass(sub.detector, sub.params, sub.n_events, d, sub.velo_x, sub.velo_y,
                           sub.velo_tx, sub.velo_ty, sub.velo_offsets)
        return int(cuts[k]), int(cuts[k + 1]), d, c

    with ThreadPoolExecutor(n) as ex:
        return list(ex.map(run, range(n)))


def test_pileup_full_every_output():
    """All 10000 pile-up events: every decoded hit, every track output and the fraction of VELO
    tracks with a candidate, against the oracle (run on event slices over the host's CPUs)."""
    b = synth.generate("pileup", with_truth=False)
    geom, dv, hits, res = _run_tuned(b)
    nh = _common_properties(b, hits, res)
    S = b.detector.n_sectors
    nb = L * S
    ho = _u32(hits["hit_offsets"]).astype(np.int64)
    n = int(ho[-1])
    h = {f: _u32(hits[f][:n]) for f in ("lhcbid", "u", "weight", "z", "y_begin", "y_end")}
    gi_all = res["hit_idx"].cpu().numpy().astype(np.int64)
    q_all, c2_all = _u32(res["qop"]), _u32(res["chi2"])
    vo = b.velo_offsets.astype(np.int64)
    found_oracle = 0
    for e0, e1, d, c in _oracle_slices(b, 16):
        g0, g1 = int(ho[e0 * nb]), int(ho[e1 * nb])
        assert np.array_equal(ho[e0 * nb:e1 * nb + 1] - g0, d["hit_offsets"].astype(np.int64)), (e0, e1)
        for f in h:
            assert np.array_equal(h[f][g0:g1], d[f][:g1 - g0].view(np.uint32)), (e0, f)
        t0, t1 = vo[e0], vo[e1]
        oi = c["hit_idx"].astype(np.int64)
        assert np.array_equal(gi_all[t0:t1], np.where(oi >= 0, oi + g0, -1)), e0
        assert np.array_equal(nh[t0:t1], c["nhits"]), e0
        assert np.array_equal(q_all[t0:t1], c["qop"].view(np.uint32)), e0
        assert np.array_equal(c2_all[t0:t1], c["chi2"].view(np.uint32)), e0
        found_oracle += int((c["nhits"] > 0).sum())
    found_gpu = int((nh > 0).sum())
    assert found_gpu == found_oracle
    print(f"[pileup full] found fraction {found_gpu / b.n_tracks:.5f} (GPU) = "
          f"{found_oracle / b.n_tracks:.5f} (oracle), {b.n_tracks} VELO tracks", flush=True)


def test_fitgrad_full_million_tracks():
    b = synth.generate("fitgrad", with_truth=False)
    geom, dv, hits, res = _run_tuned(b)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events, hit_capacity=b.n_words)
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                       b.velo_ty, b.velo_offsets)
    assert np.array_equal(res["hit_idx"].cpu().numpy(), c["hit_idx"])
    keep = c["nhits"] >= 3
    assert keep.sum() > 1_000_000
    kd = torch.from_numpy(keep).to(DEV)
    rng = np.random.default_rng(77)
    q = (c["qop"][keep].astype(np.float64) * (1 + rng.normal(0, 0.05, int(keep.sum())))).astype(np.float32)
    off = rng.normal(0, 0.05, L * b.detector.n_sectors).astype(np.float32)
    g = utc.compass_fit_grad(geom, res["hit_idx"][kd].contiguous(), hits["u"], hits["weight"],
                             hits["lhcbid"], *(v[kd].contiguous() for v in dv["vel"]),
                             torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV))
    # the same fits on the hits frozen in track-major form: identical results
    fz = utc.compass_fit_freeze(geom, res["hit_idx"][kd].contiguous(), hits["u"], hits["weight"],
                                hits["lhcbid"])
    g2 = utc.compass_fit_grad_frozen(geom, fz, *(v[kd].contiguous() for v in dv["vel"]),
                                     torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    for k, v in g2.items():
        assert np.array_equal(v.cpu().numpy().view(np.uint8), g[k].view(np.uint8)), k
    args = (b.detector, c["hit_idx"][keep], d["u"], d["weight"], d["lhcbid"], b.velo_x[keep],
            b.velo_y[keep], b.velo_tx[keep], b.velo_ty[keep])
    o = oracle.fit_grad(*args, q, off, precision="f32")
    assert np.array_equal(g["chi2_track"].view(np.uint32), o["chi2_track"].view(np.uint32))
    assert np.array_equal(g["grad_qop"].view(np.uint32), o["grad_qop"].view(np.uint32))
    # offsets: the GPU sums every term exactly in fixed point at 2^-40 (one rounding of at most
    # 2^-41 per term), the oracle in binary64; both round the sum to binary32 once
    n_terms = int((c["hit_idx"][keep] >= 0).sum())
    go, oo = g["grad_offsets"].astype(np.float64), o["grad_offsets"].astype(np.float64)
    assert np.all(np.abs(go - oo) <= np.spacing(np.abs(oo)) + n_terms * 2.0 ** -41)
    o64 = oracle.fit_grad(*args, q.astype(np.float64), off.astype(np.float64), precision="f64")
    for k in ("grad_qop", "grad_offsets", "chi2_track"):
        a, e = g[k].astype(np.float64), o64[k]
        floor = 1e-3 * np.sqrt(np.mean(e * e))
        assert np.all(np.abs(a - e) <= 1e-4 * np.abs(e) + floor), k
    assert g["chi2_total"][0] == pytest.approx(o64["chi2_total"], rel=1e-5)
