#!/usr/bin/env python3
"""Throughput of the UT chain on one MI355X: raw-bank decoding + Compass tracking + the fit-chi2
forward/backward pass, over one batch of synthetic LHCb-shaped events per step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload realistic]

Prints one JSON line.  `value` = events per second of the whole step with inputs resident in HBM.
Per-call durations come from HIP events on the stream the library launches on; the dominant call's
algorithmic bytes over its average duration give the roofline fraction against the 8 TB/s HBM peak.
The CPU baseline is the plain oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="realistic")
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--rotate", type=int, default=3,
                    help="input/output copies used round-robin so the working set exceeds the 256 MB Infinity Cache")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of HIP graph replays")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes instead of the tuned ones")
    ap.add_argument("--no-per-event", action="store_true", help="skip the one-event-at-a-time comparison")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): events are independent, so "
              "the path shards by event ranges with no exchange; multi-GPU runs are not part of "
              "this build.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2002_11529_amd as utc

    dev = torch.device("cuda:0")
    b = synth.generate(args.workload, n_events=args.events, with_truth=False)
    E, S = b.n_events, b.detector.n_sectors
    NB = E * 4 * S
    geom = utc.Geometry(b.detector, dev)
    params = utc.compass_params(b.params)
    L = utc.library()

    R = max(1, args.rotate)
    copies = []
    for _ in range(R):
        words = torch.from_numpy(b.words.view(np.int16).copy()).to(dev)
        boff = torch.from_numpy(b.bank_offsets.view(np.int32).copy()).to(dev)
        vel = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
               for a in (b.velo_x, b.velo_y, b.velo_tx, b.velo_ty)]
        vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(dev)
        cap = b.n_words
        hits = dict(hit_offsets=torch.empty(NB + 1, dtype=torch.int32, device=dev),
                    lhcbid=torch.empty(cap, dtype=torch.int32, device=dev),
                    **{k: torch.empty(cap, dtype=torch.float32, device=dev)
                       for k in ("z", "u", "y_begin", "y_end", "weight")})
        n = b.n_tracks
        res = dict(hit_idx=torch.empty((n, 4), dtype=torch.int32, device=dev),
                   qop=torch.empty(n, dtype=torch.float32, device=dev),
                   chi2=torch.empty(n, dtype=torch.float32, device=dev),
                   nhits=torch.empty(n, dtype=torch.int32, device=dev))
        fg = dict(chi2_total=torch.empty(1, dtype=torch.float64, device=dev),
                  chi2_track=torch.empty(n, dtype=torch.float32, device=dev),
                  grad_qop=torch.empty(n, dtype=torch.float32, device=dev),
                  grad_offsets=torch.empty(4 * S, dtype=torch.float32, device=dev))
        copies.append(dict(words=words, boff=boff, vel=vel, vo=vo, hits=hits, res=res, fg=fg))
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    offsets = torch.zeros(4 * S, dtype=torch.float32, device=dev)
    ws_dec = torch.empty(L.ut_decode_workspace_bytes(E, S), dtype=torch.uint8, device=dev)
    ws_find = torch.empty(max(256, L.compass_find_workspace_bytes(E, b.n_tracks)), dtype=torch.uint8, device=dev)
    ws_fg = torch.empty(L.compass_fit_grad_workspace_bytes(S), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_autotune:
        c0 = copies[0]
        tuned = utc.autotune(geom, params, E, c0["words"], c0["boff"], *c0["vel"], c0["vo"], reps=5)
    lau_dec = tuned["decode"] if tuned else None
    lau_find = tuned["find"] if tuned else None

    def step(c, ev=None):
        stream = torch.cuda.current_stream()
        if ev is not None:
            ev[0].record(stream)
        utc.ut_decode(geom, c["words"], c["boff"], E, hit_capacity=b.n_words, error_flags=flags,
                      out=c["hits"], workspace=ws_dec, launch=lau_dec)
        if ev is not None:
            ev[1].record(stream)
        utc.compass_find(geom, params, E, c["hits"], *c["vel"], c["vo"], error_flags=flags,
                         out=c["res"], workspace=ws_find, launch=lau_find)
        if ev is not None:
            ev[2].record(stream)
        utc.compass_fit_grad(geom, c["res"]["hit_idx"], c["hits"]["u"], c["hits"]["weight"],
                             c["hits"]["lhcbid"], *c["vel"], c["res"]["qop"], offsets,
                             out=c["fg"], workspace=ws_fg)
        if ev is not None:
            ev[3].record(stream)

    for i in range(args.warmup):
        step(copies[i % R])
    torch.cuda.synchronize()
    n_valid = int(copies[0]["hits"]["hit_offsets"][-1].item())
    n_found = int((copies[0]["res"]["nhits"] > 0).sum().item())
    if int(flags.item()) != 0:
        raise RuntimeError(f"device error flags {int(flags.item())}")

    # per-call durations: eager launches with HIP events between the calls
    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    for i in range(K):
        step(copies[i % R], evs[i])
    torch.cuda.synchronize()
    call_ms = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs]).mean(axis=0)

    # the step captured once per buffer copy in a HIP graph, replayed
    graphs = None
    if not args.no_graph:
        graphs = []
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for c in copies:
                gph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gph, stream=side):
                    stream = torch.cuda.current_stream()
                    step(c)
                graphs.append(gph)
        torch.cuda.current_stream().wait_stream(side)
        stream = torch.cuda.current_stream()
        for i in range(args.warmup):
            graphs[i % R].replay()
        torch.cuda.synchronize()

    # timed region: K whole steps, bracketed by synchronisation
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for i in range(K):
        if graphs is not None:
            graphs[i % R].replay()
        else:
            step(copies[i % R])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_per_step = ms_total / K
    if int(flags.item()) != 0:
        raise RuntimeError(f"device error flags {int(flags.item())}")

    # the same decode + Compass work launched one event at a time (eager), for comparison
    per_event = None
    if not args.no_per_event:
        c = copies[0]
        host_ho = c["hits"]["hit_offsets"].cpu().numpy().view(np.uint32).copy()
        hits2 = {k: torch.empty_like(v) for k, v in c["hits"].items() if k != "error_flags"}
        res2 = {k: torch.empty_like(v) for k, v in c["res"].items() if k != "error_flags"}
        scratch = utc.api.per_event_loop(geom, params, E, c["words"], c["boff"], *c["vel"], c["vo"],
                                         b.bank_offsets, host_ho, hits2, res2)
        torch.cuda.synchronize()
        pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pe0.record(stream)
        utc.api.per_event_loop(geom, params, E, c["words"], c["boff"], *c["vel"], c["vo"],
                               b.bank_offsets, host_ho, hits2, res2, scratch=scratch)
        pe1.record(stream)
        torch.cuda.synchronize()
        pe_ms = pe0.elapsed_time(pe1)
        per_event = {"events_per_s": round(E / (pe_ms * 1e-3), 1), "ms": round(pe_ms, 3),
                     "what": "ut_decode + compass_find, one event per call, eager launches"}

    # algorithmic bytes (each input read once, each output written once)
    Nw, Nh, Nt = b.n_words, n_valid, b.n_tracks
    bytes_decode = 2 * Nw + 4 * (NB + 1) + 4 * (NB + 1) + 24 * Nh
    bytes_find = 16 * Nt + 4 * (E + 1) + 28 * Nt
    fg_hits = int((copies[0]["res"]["hit_idx"] >= 0).sum().item())
    bytes_fg = Nt * (16 + 16 + 4 + 8) + fg_hits * 12 + 2 * 4 * (4 * S)
    bytes_step = 2 * Nw + 8 * NB + 24 * Nh + 44 * Nt
    names = ["ut_decode", "compass_find", "compass_fit_grad"]
    per_call_bytes = [bytes_decode, bytes_find, bytes_fg]
    dom = int(np.argmax(call_ms))
    achieved = per_call_bytes[dom] / (call_ms[dom] * 1e-3) / 1e9
    value = E / (ms_per_step * 1e-3)

    out = {
        "metric": "events/s UT decode+Compass @1 GPU (HBM GB/s); fwd+bwd fitted tracks/s",
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {E} events, {S} sectors/layer, {Nt} VELO tracks, "
                               f"{Nh} hits, {Nw} raw words",
                   "step": "ut_decode + compass_find + compass_fit_grad(fwd+bwd)",
                   "rotated_copies": R},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "calls_ms": {n: round(float(m), 5) for n, m in zip(names, call_ms)},
        "step_algorithmic_GBps": round(bytes_step / (ms_per_step * 1e-3) / 1e9, 1),
        "fitted_tracks_per_s": round(n_found / (call_ms[2] * 1e-3), 1) if call_ms[2] > 0 else None,
        "decode_GBps": round(bytes_decode / (call_ms[0] * 1e-3) / 1e9, 1),
        "timing": "hip graph replay" if graphs is not None else "eager launches",
        "launch": {"decode": lau_dec, "find": lau_find, "source": "autotuner" if tuned else "defaults"},
        "batched_vs_per_event": per_event,
        "found_fraction": round(n_found / max(Nt, 1), 5),
        "wall_s": round(wall, 4),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(b, seconds):
    """The oracle (single thread) on the same events, repeated until about `seconds` elapse."""
    import numpy as np
    import oracle
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < seconds and reps < 50:
        d = oracle.decode(b.detector, b.words, b.bank_offsets, b.n_events)
        c = oracle.compass(b.detector, b.params, b.n_events, d, b.velo_x, b.velo_y, b.velo_tx,
                           b.velo_ty, b.velo_offsets)
        oracle.fit_grad(b.detector, c["hit_idx"], d["u"], d["weight"], d["lhcbid"], b.velo_x, b.velo_y,
                        b.velo_tx, b.velo_ty, c["qop"], np.zeros(4 * b.detector.n_sectors, np.float32))
        reps += 1
        t = time.perf_counter() - t0
    return {"value": round(reps * b.n_events / t, 1), "unit": "events/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} passes over the {b.n_events}-event batch (decode + Compass + fit-chi2 "
                      f"fwd+bwd), single thread, {t:.1f} s"}


if __name__ == "__main__":
    main()
