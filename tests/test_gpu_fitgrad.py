"""GPU parity of the differentiation mode: compass_fit_grad and CompassChi2Function.

Per-track chi2 and d chi2/d qop follow the same float32 operation sequence as the oracle and must
match it bit for bit; the offset gradients and the total are exact integer sums on the GPU and
binary64 sums in the oracle, so they may differ in the last bit.  Against the binary64 reference
gradient the tolerance is 1e-4 relative (component-wise, with a floor of 1e-3 of the RMS), and
against central finite differences of the GPU's own chi2 (h = 1e-3 mm) 1e-3 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frozen():
    b = synth.generate("fitgrad", n_events=400, with_truth=False)
    print(f"[fitgrad frozen] events={b.n_events} tracks={b.n_tracks}", flush=True)
    h, r, geom, hits, res, dv = gpu_run(b)
    d, c = oracle_run(b)
    keep = c["nhits"] >= 3
    # the GPU's frozen assignment is the oracle's (bit-exact parity of the search)
    assert np.array_equal(r["hit_idx"], c["hit_idx"])
    kd = torch.from_numpy(keep).to(DEV)
    F = dict(track_hit_idx=res["hit_idx"][kd].contiguous(), hit_u=hits["u"], hit_weight=hits["weight"],
             hit_lhcbid=hits["lhcbid"],
             **{k: v[kd].contiguous() for k, v in zip(("vx", "vy", "vtx", "vty"), dv["vel"])})
    return dict(b=b, d=d, geom=geom, F=F, keep=keep, qop=res["qop"][kd].contiguous(),
                idx=c["hit_idx"][keep], qop_np=c["qop"][keep])


def _gpu(fr, qop, off, scale=1.0):
    F = fr["F"]
    r = utc.compass_fit_grad(fr["geom"], F["track_hit_idx"], F["hit_u"], F["hit_weight"], F["hit_lhcbid"],
                             F["vx"], F["vy"], F["vtx"], F["vty"], qop, off, grad_scale=scale)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _ora(fr, qop, off, precision, scale=1.0):
    b, d, k = fr["b"], fr["d"], fr["keep"]
    return oracle.fit_grad(b.detector, fr["idx"], d["u"], d["weight"], d["lhcbid"], b.velo_x[k],
                           b.velo_y[k], b.velo_tx[k], b.velo_ty[k], qop, off, grad_scale=scale,
                           precision=precision)


def _point(fr, seed):
    rng = np.random.default_rng(seed)
    q = (fr["qop_np"].astype(np.float64) * (1 + rng.normal(0, 0.05, fr["qop_np"].shape[0]))).astype(np.float32)
    off = rng.normal(0, 0.05, 800).astype(np.float32)
    return q, off


def test_matches_float32_oracle(frozen):
    q, off = _point(frozen, 1)
    g = _gpu(frozen, torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV), scale=0.75)
    o = _ora(frozen, q, off, "f32", scale=0.75)
    assert np.array_equal(g["chi2_track"].view(np.uint32), o["chi2_track"].view(np.uint32))
    assert np.array_equal(g["grad_qop"].view(np.uint32), o["grad_qop"].view(np.uint32))
    go, oo = g["grad_offsets"], o["grad_offsets"]
    ulp = np.spacing(np.abs(oo)).astype(np.float64)
    assert np.all(np.abs(go.astype(np.float64) - oo) <= ulp)
    assert g["chi2_total"][0] == pytest.approx(o["chi2_total"], rel=1e-12)


def test_matches_float64_reference(frozen):
    q, off = _point(frozen, 2)
    g = _gpu(frozen, torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV))
    o = _ora(frozen, q.astype(np.float64), off.astype(np.float64), "f64")
    for k in ("grad_qop", "grad_offsets", "chi2_track"):
        a, e = g[k].astype(np.float64), o[k]
        floor = 1e-3 * np.sqrt(np.mean(e * e))
        assert np.all(np.abs(a - e) <= 1e-4 * np.abs(e) + floor), k
    assert g["chi2_total"][0] == pytest.approx(o["chi2_total"], rel=1e-5)


def test_matches_central_differences(frozen):
    q, off = _point(frozen, 3)
    qd, od = torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV)
    base = _gpu(frozen, qd, od)
    S = 200
    lid = frozen["d"]["lhcbid"]
    fd = np.zeros(800)
    h = 1e-3
    for l in range(4):
        p = off.copy(); p[l * S:(l + 1) * S] += np.float32(h)
        m = off.copy(); m[l * S:(l + 1) * S] -= np.float32(h)
        cp = _gpu(frozen, qd, torch.from_numpy(p).to(DEV))["chi2_track"].astype(np.float64)
        cm = _gpu(frozen, qd, torch.from_numpy(m).to(DEV))["chi2_track"].astype(np.float64)
        step = (p[l * S:(l + 1) * S].astype(np.float64) - m[l * S:(l + 1) * S].astype(np.float64))
        hl = frozen["idx"][:, l]
        has = hl >= 0
        sec = ((lid[hl[has]].astype(np.int64) >> 12) & 0xFFFF)
        np.add.at(fd, l * S + sec, (cp - cm)[has] / step[sec])
    go = base["grad_offsets"].astype(np.float64)
    used = go != 0
    floor = 1e-3 * np.sqrt(np.mean(go[used] ** 2))
    assert np.all(np.abs(fd - go) <= 1e-3 * np.abs(go) + floor)
    # q/p: perturb all tracks at once (they are independent)
    hq = np.float32(1e-3 / 1200.0)
    qp, qm = q + hq, q - hq
    cp = _gpu(frozen, torch.from_numpy(qp).to(DEV), od)["chi2_track"].astype(np.float64)
    cm = _gpu(frozen, torch.from_numpy(qm).to(DEV), od)["chi2_track"].astype(np.float64)
    fdq = (cp - cm) / (qp.astype(np.float64) - qm.astype(np.float64))
    gq = base["grad_qop"].astype(np.float64)
    floor = 1e-3 * np.sqrt(np.mean(gq ** 2))
    assert np.all(np.abs(fdq - gq) <= 1e-3 * np.abs(gq) + floor)


def test_forward_only_and_repeatability(frozen):
    q, off = _point(frozen, 4)
    qd, od = torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV)
    F = frozen["F"]
    r1 = utc.compass_fit_grad(frozen["geom"], F["track_hit_idx"], F["hit_u"], F["hit_weight"],
                              F["hit_lhcbid"], F["vx"], F["vy"], F["vtx"], F["vty"], qd, od,
                              want_grad=False, want_chi2_track=False)
    a = _gpu(frozen, qd, od)
    b2 = _gpu(frozen, qd, od)
    torch.cuda.synchronize()
    assert float(r1["chi2_total"][0]) == a["chi2_total"][0]
    for k in a:
        assert a[k].tobytes() == b2[k].tobytes()


def test_autograd_function(frozen):
    q, off = _point(frozen, 5)
    qd = torch.from_numpy(q).to(DEV).requires_grad_(True)
    od = torch.from_numpy(off).to(DEV).requires_grad_(True)
    chi2 = utc.CompassChi2Function.apply(qd, od, frozen["geom"], frozen["F"])
    (2.0 * chi2).backward()
    ref = _gpu(frozen, qd.detach(), od.detach(), scale=2.0)
    assert float(chi2.detach()) == ref["chi2_total"][0]
    assert np.allclose(qd.grad.cpu().numpy(), ref["grad_qop"], rtol=1e-6, atol=0)
    assert np.allclose(od.grad.cpu().numpy(), ref["grad_offsets"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("seed", [3, 4])
def test_frozen_layout_equals_gathered(frozen, seed):
    """compass_fit_freeze + compass_fit_grad_frozen give the gathered call's results bit for bit,
    including tracks with 3 hits and slots that the gathered call skips (index -1, out of range)."""
    fr = frozen
    F = fr["F"]
    q, off = _point(fr, seed)
    qd, od = torch.from_numpy(q).to(DEV), torch.from_numpy(off).to(DEV)
    idx = F["track_hit_idx"].clone()
    n = int(idx.shape[0])
    # a few slots the gathered call skips
    idx[5, 1] = -1
    idx[7, 2] = int(F["hit_u"].shape[0]) + 3
    ref = utc.compass_fit_grad(fr["geom"], idx, F["hit_u"], F["hit_weight"], F["hit_lhcbid"], F["vx"],
                               F["vy"], F["vtx"], F["vty"], qd, od)
    fz = utc.compass_fit_freeze(fr["geom"], idx, F["hit_u"], F["hit_weight"], F["hit_lhcbid"])
    got = utc.compass_fit_grad_frozen(fr["geom"], fz, F["vx"], F["vy"], F["vtx"], F["vty"], qd, od)
    torch.cuda.synchronize()
    ts = fz["track_sector"].cpu().numpy()
    assert ts[5, 1] == -1 and ts[7, 2] == -1 and (ts[:, 0] >= 0).sum() > 0.9 * n
    for k in ("chi2_track", "grad_qop", "grad_offsets", "chi2_total"):
        a, e = got[k].cpu().numpy(), ref[k].cpu().numpy()
        assert np.array_equal(a.view(np.uint8), e.view(np.uint8)), k
