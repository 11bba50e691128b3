"""Steps on several streams at once: batches of different shapes decoded, searched and
differentiated concurrently, each on its own stream with its own outputs and workspaces, give bit
for bit what the same calls give one after another (the library keeps no state between calls; the
error-flag word is only OR-ed)."""
import numpy as np
import pytest
import torch

import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu

BATCHES = [("realistic", 300, 11), ("realistic", 300, 12), ("batched", 200, 13)]


def _step(geom, b, dv, offsets):
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events)
    res = utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"])
    fg = utc.compass_fit_grad(geom, res["hit_idx"], hits["u"], hits["weight"], hits["lhcbid"], *dv["vel"],
                              res["qop"], offsets)
    return hits, res, fg


def _host(out):
    hits, res, fg = out
    n = int(hits["hit_offsets"][-1])
    h = {k: (v if k in ("hit_offsets", "error_flags") else v[:n]).cpu().numpy() for k, v in hits.items()}
    return h, {k: v.cpu().numpy() for k, v in res.items()}, {k: v.cpu().numpy() for k, v in fg.items()}


def _same(a, b, what):
    for x, y in zip(a, b):
        assert x.keys() == y.keys()
        for k in x:
            assert np.array_equal(x[k].view(np.uint8), y[k].view(np.uint8)), f"{what}: {k}"


def test_concurrent_steps_match_sequential():
    work = []
    for name, n, seed in BATCHES:
        b = synth.generate(name, n_events=n, seed=seed, with_truth=False)
        geom = utc.Geometry(b.detector, DEV)
        offsets = torch.from_numpy(
            np.random.default_rng(seed).normal(0, 0.05, 4 * b.detector.n_sectors).astype(np.float32)).to(DEV)
        work.append((geom, b, to_dev(b), offsets))
    print(f"[streams] batches={[(n, w[1].n_events, w[1].n_tracks) for n, w in zip(BATCHES, work)]}", flush=True)
    ref = [_host(_step(*w)) for w in work]
    torch.cuda.synchronize()
    for i, r in enumerate(ref):
        assert r[0]["error_flags"][0] == 0 and r[1]["error_flags"][0] == 0
        assert (r[1]["nhits"] > 0).mean() > 0.5, i

    streams = [torch.cuda.Stream() for _ in work]
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):   # three rounds, each launching every batch on its own stream
        for st, w in zip(streams, work):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                outs.append(_step(*w))
    for st in streams:
        torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    for j, o in enumerate(outs):
        _same(_host(o), ref[j % len(work)], f"round {j // len(work)}, batch {BATCHES[j % len(work)]}")


def test_full_size_graph_replays_on_three_streams():
    """The realistic batch at full size as the benchmark times it: autotuned launch shapes, the
    step captured in a HIP graph per buffer copy, the graphs replayed on three streams at once
    (twice); every copy's decoded hits and tracks equal the oracle's bit for bit."""
    from tests.gpu_helpers import oracle_run, assert_decode_equal, assert_compass_equal
    b = synth.generate("realistic", with_truth=False)
    E = b.n_events
    geom = utc.Geometry(b.detector, DEV)
    L = utc.library()
    copies = [dict(dv=to_dev(b)) for _ in range(3)]
    dv0 = copies[0]["dv"]
    t = utc.autotune(geom, b.params, E, dv0["words"], dv0["bank_offsets"], *dv0["vel"], dv0["velo_offsets"])
    print(f"[streams full] events={E} tracks={b.n_tracks} launch={t['decode']} {t['find']}", flush=True)
    for c in copies:
        dv = c["dv"]
        c["wd"] = torch.empty(L.ut_decode_workspace_bytes(E, b.detector.n_sectors), dtype=torch.uint8, device=DEV)
        c["wf"] = torch.empty(max(256, L.compass_find_workspace_bytes(E, b.n_tracks)), dtype=torch.uint8,
                              device=DEV)
        c["hits"] = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], E, launch=t["decode"], workspace=c["wd"])
        c["res"] = utc.compass_find(geom, b.params, E, c["hits"], *dv["vel"], dv["velo_offsets"],
                                    launch=t["find"], workspace=c["wf"])
    torch.cuda.synchronize()
    for c in copies:   # the replays must write every output again
        for k, v in c["hits"].items():
            if k != "error_flags":
                v.fill_(-1)
        for k in ("hit_idx", "qop", "chi2", "nhits"):
            c["res"][k].fill_(-7)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graphs = []
    with torch.cuda.stream(side):
        for c in copies:
            dv = c["dv"]
            gph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gph, stream=side):
                utc.ut_decode(geom, dv["words"], dv["bank_offsets"], E, error_flags=c["hits"]["error_flags"],
                              out=c["hits"], workspace=c["wd"], launch=t["decode"])
                utc.compass_find(geom, b.params, E, c["hits"], *dv["vel"], dv["velo_offsets"],
                                 error_flags=c["res"]["error_flags"], out=c["res"], workspace=c["wf"],
                                 launch=t["find"])
            graphs.append(gph)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in copies]
    for _ in range(2):
        for st, gph in zip(streams, graphs):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                gph.replay()
    for st in streams:
        torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    d, o = oracle_run(b)
    for i, c in enumerate(copies):
        h = {k: v.cpu().numpy() for k, v in c["hits"].items()}
        h["hit_offsets"] = h["hit_offsets"].view(np.uint32)
        h["lhcbid"] = h["lhcbid"].view(np.uint32)
        assert int(h["error_flags"][0]) == 0 and int(c["res"]["error_flags"][0]) == 0, i
        assert_decode_equal(h, d)
        assert_compass_equal({k: v.cpu().numpy() for k, v in c["res"].items()}, o)
