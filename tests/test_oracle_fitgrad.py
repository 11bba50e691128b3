"""Pins of the oracle track-fit chi2 and its adjoint (the differentiation mode).

chi2 is exactly quadratic in q/p and in the per-sector offsets, so a central finite difference is
exact up to rounding: the float64 adjoint must match it to ~1e-9.  At the fitted q/p of the
tracklet search and zero offsets, the chi2 equals the search's own chi2 bit for bit and its q/p
derivative vanishes (the fit is a least-squares minimum).
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def frozen():
    b = synth.generate("fitgrad", n_events=40)
    d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
    c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                       b.velo_ty, b.velo_offsets)
    keep = c["nhits"] >= 3
    return dict(b=b, d=d, c=c, keep=keep, idx=c["hit_idx"][keep],
                vel=[a[keep] for a in (b.velo_x, b.velo_y, b.velo_tx, b.velo_ty)],
                qop=c["qop"][keep], chi2=c["chi2"][keep])


def _fg(fr, qop, off, precision="f64", scale=1.0):
    d = fr["d"]
    return oracle.fit_grad(fr["b"].detector, fr["idx"], d["u"], d["weight"], d["lhcbid"], *fr["vel"],
                           qop, off, grad_scale=scale, precision=precision)


def test_chi2_matches_search_chi2_at_fit(frozen):
    """At zero offsets and the search's q/p the fit chi2 is the search's selection chi2; they differ
    only by the float32 cancellation in the search's residuals."""
    off = np.zeros(4 * 200, np.float32)
    r = _fg(frozen, frozen["qop"], off, "f32")
    assert np.allclose(r["chi2_track"], frozen["chi2"], rtol=2e-2, atol=2e-3)
    assert r["chi2_total"] == pytest.approx(float(frozen["chi2"].astype(np.float64).sum()), rel=1e-3)
    assert r["chi2_total"] == pytest.approx(float(r["chi2_track"].astype(np.float64).sum()), rel=1e-12)


def test_qop_gradient_vanishes_at_least_squares_minimum(frozen):
    """d chi2/d qop = -2 (S_ar - qop S_aa) is zero at the fitted qop, up to the float32 rounding
    of the residuals the search's fit was computed from."""
    off = np.zeros(4 * 200)
    r = _fg(frozen, frozen["qop"].astype(np.float64), off)
    det = frozen["b"].detector
    d = frozen["d"]
    x, y, tx, ty = [v.astype(np.float64) for v in frozen["vel"]]
    bound = np.zeros(x.shape[0])
    saa = np.zeros(x.shape[0])
    for l in range(4):
        h = frozen["idx"][:, l]
        has = h >= 0
        dz = float(det.z_layer[l]) - float(det.z_velo)
        a = float(det.a_kick[l])
        w = np.where(has, d["weight"][h], 0.0)
        mag = np.abs(d["u"][h]) + np.abs(x + tx * dz) + np.abs((y + ty * dz) * float(det.dxdy[l]))
        bound += 2 * w * a * 8 * 2.0 ** -24 * np.where(has, mag, 0.0)
        saa += w * a * a
    bound += 2 * saa * 2.0 ** -23 * np.abs(frozen["qop"])
    g = r["grad_qop"]
    assert np.all(np.abs(g) <= bound)
    # the bound is far below the size of the individual terms
    assert np.median(bound) < 1e-2 * np.median(2 * saa * np.abs(frozen["qop"]))


def _point(fr, seed):
    rng = np.random.default_rng(seed)
    qop = fr["qop"].astype(np.float64) * (1 + rng.normal(0, 0.05, fr["qop"].shape[0]))
    off = rng.normal(0, 0.05, 800)
    return qop, off


def test_gradient_matches_central_differences_f64(frozen):
    qop, off = _point(frozen, 1)
    base = _fg(frozen, qop, off)
    # q/p: tracks are independent, so perturb all of them at once and read per-track chi2
    h = 1e-3 / 1200.0
    cp = _fg(frozen, qop + h, off)["chi2_track"]
    cm = _fg(frozen, qop - h, off)["chi2_track"]
    fd = (cp - cm) / (2 * h)
    g = base["grad_qop"]
    assert np.allclose(fd, g, rtol=1e-7, atol=1e-9 * np.abs(g).max())
    # offsets: a track touches one sector per layer, so perturb one layer's sectors together and
    # attribute each track's chi2 change to the sector of its hit in that layer
    S = 200
    lid = frozen["d"]["lhcbid"]
    fd_off = np.zeros(800)
    hd = 1e-3
    for l in range(4):
        p = off.copy(); p[l * S:(l + 1) * S] += hd
        m = off.copy(); m[l * S:(l + 1) * S] -= hd
        dc = (_fg(frozen, qop, p)["chi2_track"] - _fg(frozen, qop, m)["chi2_track"]) / (2 * hd)
        h_l = frozen["idx"][:, l]
        has = h_l >= 0
        sec = l * S + ((lid[h_l[has]].astype(np.int64) >> 12) & 0xFFFF)
        np.add.at(fd_off, sec, dc[has])
    go = base["grad_offsets"]
    assert np.abs(go).max() > 0
    assert np.allclose(fd_off, go, rtol=1e-7, atol=1e-9 * np.abs(go).max())


def test_f32_adjoint_close_to_f64(frozen):
    qop, off = _point(frozen, 2)
    r64 = _fg(frozen, qop, off, "f64", scale=0.5)
    r32 = _fg(frozen, qop.astype(np.float32), off.astype(np.float32), "f32", scale=0.5)
    for k in ("grad_qop", "grad_offsets", "chi2_track"):
        a, b = r32[k].astype(np.float64), r64[k]
        floor = 1e-3 * np.sqrt(np.mean(b * b))
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + floor), k
    assert r32["chi2_total"] == pytest.approx(r64["chi2_total"], rel=1e-5)


def test_grad_scale_is_linear(frozen):
    qop, off = _point(frozen, 3)
    r1 = _fg(frozen, qop, off, scale=1.0)
    r3 = _fg(frozen, qop, off, scale=-3.0)
    assert np.allclose(r3["grad_qop"], -3 * r1["grad_qop"], rtol=1e-12)
    assert np.allclose(r3["grad_offsets"], -3 * r1["grad_offsets"], rtol=1e-12)
    assert np.array_equal(r3["chi2_track"], r1["chi2_track"])


def test_misalignment_signal_in_gradient(frozen):
    """With hits displaced by the hidden offsets, the offset gradient at zero points against them."""
    b = frozen["b"]
    det = b.detector
    r = _fg(frozen, frozen["qop"].astype(np.float64), np.zeros(800))
    g = r["grad_offsets"]
    used = g != 0
    # d chi2/d delta_s = -2 sum w (r - delta): residuals carry +delta_true, so the gradient is
    # negatively correlated with delta_true on well-populated sectors
    corr = np.corrcoef(g[used], b.delta_true[used])[0, 1]
    assert corr < -0.3, corr
