"""The batched path: many uneven events in one launch (direct, persistent, autotuned, and replayed
from a HIP graph) gives the same bytes as the same work launched one event at a time."""
import numpy as np
import pytest
import torch

import synth
import paper_2002_11529_amd as utc
from tests.gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uneven():
    b = synth.generate("batched", n_events=60, seed=33, with_truth=False)
    print(f"[batched 60] words={b.n_words} tracks={b.n_tracks} "
          f"tracks/event {np.diff(b.velo_offsets.astype(np.int64)).min()}.."
          f"{np.diff(b.velo_offsets.astype(np.int64)).max()}", flush=True)
    return b, to_dev(b), utc.Geometry(b.detector, DEV)


def _batched(b, dv, geom, launch_decode=None, launch_find=None):
    hits = utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, launch=launch_decode)
    res = utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"],
                           launch=launch_find)
    torch.cuda.synchronize()
    return hits, res


def test_batched_equals_per_event_loop(uneven):
    b, dv, geom = uneven
    hits, res = _batched(b, dv, geom)
    host_ho = hits["hit_offsets"].cpu().numpy().view(np.uint32)
    n = int(host_ho[-1])
    cap = b.n_words
    hits2 = {k: torch.zeros_like(hits[k]) for k in ("lhcbid", "z", "u", "y_begin", "y_end", "weight")}
    res2 = {k: torch.zeros_like(res[k]) for k in ("hit_idx", "qop", "chi2", "nhits")}
    utc.api.per_event_loop(geom, b.params, b.n_events, dv["words"], dv["bank_offsets"], *dv["vel"],
                           dv["velo_offsets"], b.bank_offsets, host_ho, hits2, res2)
    torch.cuda.synchronize()
    for k in ("lhcbid", "z", "u", "y_begin", "y_end", "weight"):
        assert torch.equal(hits[k][:n], hits2[k][:n]), k
    # per-event hit indices are relative to the event's first hit
    ev = np.repeat(np.arange(b.n_events), np.diff(b.velo_offsets.astype(np.int64)))
    base = host_ho[ev * 4 * b.detector.n_sectors].astype(np.int64)[:, None]
    idx2 = res2["hit_idx"].cpu().numpy().astype(np.int64)
    idx2 = np.where(idx2 >= 0, idx2 + base, -1)
    assert np.array_equal(res["hit_idx"].cpu().numpy(), idx2)
    for k in ("qop", "chi2", "nhits"):
        assert torch.equal(res[k], res2[k]), k


def test_persistent_shapes_equal(uneven):
    b, dv, geom = uneven
    h0, r0 = _batched(b, dv, geom)
    n = int(h0["hit_offsets"][-1])
    for ld, lf in ((dict(block=128, grid=5), dict(block=64, grid=3)),
                   (dict(block=512, grid=256), dict(block=256, grid=1024)),
                   (dict(block=64), dict(block=512)), (dict(block=256), dict(block=512, grid=7)),
                   # LDS tiles per wavefront: small chunks and window caches, large ones
                   (dict(block=256, tile=4), dict(block=256, tile=4)),
                   (dict(block=128, grid=7, tile=6), dict(block=512, grid=9, tile=8)),
                   (dict(block=256, tile=16), dict(block=256, tile=24)),
                   (dict(block=64, tile=40), dict(block=128, grid=5, tile=40))):
        h1, r1 = _batched(b, dv, geom, ld, lf)
        assert torch.equal(h0["hit_offsets"], h1["hit_offsets"])
        assert torch.equal(h0["u"][:n], h1["u"][:n]) and torch.equal(h0["lhcbid"][:n], h1["lhcbid"][:n])
        for k in ("hit_idx", "qop", "chi2", "nhits"):
            assert torch.equal(r0[k], r1[k]), k


def test_autotune_choice_is_valid_and_equal(uneven, tmp_path, monkeypatch):
    b, dv, geom = uneven
    monkeypatch.setenv("UTC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    t = utc.autotune(geom, b.params, b.n_events, dv["words"], dv["bank_offsets"], *dv["vel"],
                     dv["velo_offsets"], reps=2)
    assert t["decode"]["block"] in (64, 128, 256, 512) and t["find"]["block"] in (64, 128, 256, 512)
    assert t["decode_us"] > 0 and t["find_us"] > 0
    again = utc.autotune(geom, b.params, b.n_events, dv["words"], dv["bank_offsets"], *dv["vel"],
                         dv["velo_offsets"], reps=2)
    assert again == t   # served from the cache
    h0, r0 = _batched(b, dv, geom)
    h1, r1 = _batched(b, dv, geom, t["decode"], t["find"])
    n = int(h0["hit_offsets"][-1])
    assert torch.equal(h0["u"][:n], h1["u"][:n])
    for k in ("hit_idx", "qop", "chi2", "nhits"):
        assert torch.equal(r0[k], r1[k]), k


def test_graph_replays_match_eager(uneven):
    """decode + Compass captured once, replayed several times with eager work in between."""
    b, dv, geom = uneven
    h_ref, r_ref = _batched(b, dv, geom)
    n = int(h_ref["hit_offsets"][-1])
    hits = {k: torch.empty_like(v) for k, v in h_ref.items() if k != "error_flags"}
    res = {k: torch.empty_like(v) for k, v in r_ref.items() if k != "error_flags"}
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    L = utc.library()
    wsd = torch.empty(L.ut_decode_workspace_bytes(b.n_events, b.detector.n_sectors), dtype=torch.uint8, device=DEV)
    wsf = torch.empty(256, dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, error_flags=flags,
                          out=hits, workspace=wsd)
            utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"],
                             error_flags=flags, out=res, workspace=wsf)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for k, v in list(hits.items()) + list(res.items()):
            if k != "error_flags":
                v.fill_(-7)
        _batched(b, dv, geom)          # eager work between the replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(hits["hit_offsets"], h_ref["hit_offsets"]), rep
        assert torch.equal(hits["u"][:n], h_ref["u"][:n]), rep
        for k in ("hit_idx", "qop", "chi2", "nhits"):
            assert torch.equal(res[k], r_ref[k]), (rep, k)
    assert int(flags.item()) == 0


@pytest.mark.parametrize("tile", [0, 24])
def test_graph_replays_persistent_counter(uneven, tile):
    """A persistent Compass launch (its event counter is reset by a kernel inside the captured
    graph) replayed several times, and a second graph with its own workspace replayed on another
    stream, each against the eager result."""
    b, dv, geom = uneven
    lf = dict(block=256, grid=7, tile=tile)
    h_ref, r_ref = _batched(b, dv, geom)
    L = utc.library()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    graphs, outs = [], []
    for st in streams:
        hits = {k: torch.empty_like(v) for k, v in h_ref.items() if k != "error_flags"}
        res = {k: torch.empty_like(v) for k, v in r_ref.items() if k != "error_flags"}
        flags = torch.zeros(1, dtype=torch.int32, device=DEV)
        wsd = torch.empty(L.ut_decode_workspace_bytes(b.n_events, b.detector.n_sectors),
                          dtype=torch.uint8, device=DEV)
        wsf = torch.empty(256, dtype=torch.uint8, device=DEV)
        st.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(st):
            with torch.cuda.graph(graph, stream=st):
                utc.ut_decode(geom, dv["words"], dv["bank_offsets"], b.n_events, error_flags=flags,
                              out=hits, workspace=wsd, launch=dict(block=128, grid=9, tile=tile))
                utc.compass_find(geom, b.params, b.n_events, hits, *dv["vel"], dv["velo_offsets"],
                                 error_flags=flags, out=res, workspace=wsf, launch=lf)
        torch.cuda.current_stream().wait_stream(st)
        graphs.append(graph)
        outs.append((hits, res, flags))
    n = int(h_ref["hit_offsets"][-1])
    for rep in range(3):
        for hits, res, _ in outs:
            for k, v in list(hits.items()) + list(res.items()):
                if k != "error_flags":   # the flag word is OR-ed into, never cleared, by the calls
                    v.fill_(-7)
        torch.cuda.synchronize()
        _batched(b, dv, geom)          # eager work between the replays
        for st, graph in zip(streams, graphs):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                graph.replay()
        torch.cuda.synchronize()
        for hits, res, flags in outs:
            assert torch.equal(hits["hit_offsets"], h_ref["hit_offsets"]), rep
            assert torch.equal(hits["u"][:n], h_ref["u"][:n]), rep
            for k in ("hit_idx", "qop", "chi2", "nhits"):
                assert torch.equal(res[k], r_ref[k]), (rep, k)
            assert int(flags.item()) == 0
