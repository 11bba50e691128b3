#!/usr/bin/env python3
"""Throughput of the UT chain on one MI355X: raw-bank decoding + Compass tracking + the fit-chi2
forward/backward pass, over one batch of synthetic LHCb-shaped events per step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched] [--also realistic,pileup]

Prints one JSON line.  `value` = events per second of the whole step with inputs resident in HBM,
on the batch of 20000 events of uneven size (the largest one-GPU workload with the default window);
the realistic and pile-up workloads are timed the same way and reported as extra keys.
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
# VALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 vector instruction per SIMD every 4 cycles
# (16 lanes per SIMD), at the 2.4 GHz peak engine clock
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
KERNEL_OF_CALL = {"ut_decode": "k_decode", "compass_find": "k_compass", "compass_fit_grad": "k_fitgrad"}
# sources each kernel is compiled from: counters taken before a change to any of them no longer apply
KERNEL_SOURCES = {
    "k_compass": ["paper_2002_11529_amd/csrc/compass.hip", "paper_2002_11529_amd/csrc/compass_group.hpp",
                  "paper_2002_11529_amd/csrc/common.hpp", "include/ut_compass.h"],
    "k_decode": ["paper_2002_11529_amd/csrc/decode.hip", "paper_2002_11529_amd/csrc/decode_unit.hpp",
                 "paper_2002_11529_amd/csrc/common.hpp", "include/ut_compass.h"],
    "k_fitgrad": ["paper_2002_11529_amd/csrc/fitgrad.hip", "paper_2002_11529_amd/csrc/common.hpp",
                  "include/ut_compass.h"],
}


def kernel_source_hash(kernel):
    """Hash of the code (comments and whitespace removed) of the sources a kernel is built from."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def launch_tag(launch, n_items=None, items_per_workgroup=1):
    """The launch shape as the counter summaries record it.  A persistent grid with a workgroup
    for every work item maps the work exactly as one workgroup per item does, so both have one
    tag."""
    if not launch:
        return "defaults"
    g = launch["grid"]
    if g == 0 or (n_items is not None and g * items_per_workgroup >= n_items):
        g = "per-item"
    tag = f"block={launch['block']} grid={g}"
    if "tile" in launch:   # LDS KiB per wavefront (0: the default 10)
        tag += f" tile={launch['tile'] or 10}"
    return tag


def counter_fields(kernel, workload, what, launch=None):
    """Fields of the committed counter summary profiles/{workload}_{what}_counters.txt, or None
    when there is none, or it was taken from other kernel sources than the current ones, or (for
    an autotuned kernel) at another launch shape (`launch`, a launch_tag): a kernel's cache
    behaviour, and so its HBM traffic, depends on how many events are in flight at once."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{what}_counters.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get(f"{kernel}.source_sha256_16") != kernel_source_hash(kernel):
        return None
    if f"{kernel}.launch" in fields and fields[f"{kernel}.launch"] != launch:
        return None
    return fields


def measured_traffic(kernel, workload, launch=None):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, each scaled by what it reads for a
    plain copy of known size), or None (no summary, or one of other kernel sources or shape)."""
    fields = counter_fields(kernel, workload, "hbm", launch)
    try:
        return int(fields[f"{kernel}.hbm_bytes_per_launch"]) if fields else None
    except (KeyError, ValueError):
        return None


def measured_valu(kernel, workload, launch=None):
    """Vector-ALU instructions (wave64) per launch of `kernel` (SQ_INSTS_VALU), or None."""
    fields = counter_fields(kernel, workload, "sq", launch)
    try:
        return int(fields[f"{kernel}.valu_instr_per_launch"]) if fields else None
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched",
                    help="the workload of the headline figure (batched: 20000 uneven events)")
    ap.add_argument("--also", default="realistic,pileup",
                    help="comma-separated further workloads timed the same way (extra keys of the line)")
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--rotate", type=int, default=3,
                    help="input/output copies used round-robin so the working set exceeds the 256 MB Infinity Cache")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of HIP graph replays")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-events", type=int, default=2000,
                    help="events of the headline workload the CPU oracle is timed on")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes instead of the tuned ones")
    ap.add_argument("--no-per-event", action="store_true", help="skip the one-event-at-a-time comparison")
    ap.add_argument("--streams", type=int, default=0,
                    help="consecutive steps go to this many streams in turn (independent batches in flight "
                         "at once); every buffer copy stays on one stream.  0: each of 1, 2 and 3 streams "
                         "is timed over a short burst first and the fastest is used")
    ap.add_argument("--no-copy-bandwidth", action="store_true",
                    help="skip the 1 GiB device copy that measures the card's streaming bandwidth")
    ap.add_argument("--no-compact", action="store_true",
                    help="skip the step timed on the compact hit form (no per-hit z / y range)")
    ap.add_argument("--no-fitgrad", action="store_true",
                    help="skip the fit-chi2 forward/backward figure on the 1e6-track workload")
    ap.add_argument("--sweep", action="store_true",
                    help="only the 1/3/5-sector x 1..16-candidate sweep of compass_find: events/s and the "
                         "physics-efficiency figures on truth, one JSON line per configuration")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): events are independent, so "
              "the path shards by event ranges with no exchange; multi-GPU runs are not "
              "supported.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        copy_calibration()
        return
    if args.sweep:
        sweep(args)
        return

    head = measure_chain(args, args.workload, full=True)
    b, E, S, Nt = head["batch"], head["E"], head["S"], head["Nt"]
    copy_bw = None if args.no_copy_bandwidth else copy_bandwidth()
    dom = head["dominant"]
    kern = KERNEL_OF_CALL[dom]
    achieved = head["per_call_GBps"][dom]
    out = {
        "metric": "events/s UT decode+Compass @1 GPU (HBM GB/s); fwd+bwd fitted tracks/s",
        "value": round(head["value"], 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"],
                   "step": "ut_decode + compass_find + compass_fit_grad(fwd+bwd)",
                   "rotated_copies": head["rotated_copies"], "streams": head["streams"],
                   "search_launch_timed": head["search_launch_timed"],
                   "stream_trials_ms_per_step": head["stream_trials"]},
        "roofline": {"bound": "hbm", "kernel": kern, "call": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kern, args.workload, head["shape_tags"].get(kern)),
                     "copy_GBps": round(copy_bw, 1) if copy_bw else None,
                     "frac_of_copy": round(achieved / copy_bw, 4) if copy_bw else None,
                     "valu_issue": valu_issue(kern, args.workload, head["calls_ms"][dom],
                                              head["shape_tags"].get(kern))},
        "calls_ms": {n: round(float(m), 5) for n, m in head["calls_ms"].items()},
        "calls_algorithmic_GBps": {n: round(v, 1) for n, v in head["per_call_GBps"].items()},
        "step_algorithmic_GBps": round(head["step_GBps"], 1),
        "timing": head["timing"],
        "launch": head["launch"],
        "batched_vs_per_event": head["per_event"],
        "compact_hits": head["compact"],
        "found_fraction": round(head["found_fraction"], 5),
        "wall_s": round(head["wall_s"], 4),
    }
    out["event_cut_and_consolidation"] = head["select"]
    head = None
    torch.cuda.empty_cache()
    # the other synthetic workloads, timed the same way (graph replay, tuned shapes, best stream
    # count), without the per-event and compact comparisons
    others = {}
    for wl in [w for w in args.also.split(",") if w and w != args.workload]:
        r = measure_chain(args, wl, full=False)
        others[wl] = {"workload": r["workload"], "events_per_s": round(r["value"], 1),
                      "ms_per_step": round(r["ms_per_step"], 5), "streams": r["streams"],
                      "calls_ms": {n: round(float(m), 5) for n, m in r["calls_ms"].items()},
                      "calls_algorithmic_GBps": {n: round(v, 1) for n, v in r["per_call_GBps"].items()},
                      "step_algorithmic_GBps": round(r["step_GBps"], 1),
                      "step_frac_of_hbm_peak": round(r["step_GBps"] / HBM_PEAK_GBS, 4),
                      "found_fraction": round(r["found_fraction"], 5), "launch": r["launch"]}
        r = None
        torch.cuda.empty_cache()
    out["other_workloads"] = others
    if not args.no_fitgrad:
        out["fitgrad"] = bench_fitgrad(args, torch.device("cuda:0"))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_seconds, args.cpu_events)
    print(json.dumps(out), flush=True)


def measure_chain(args, workload, full):
    """One workload: decode + Compass + fit-chi2 fwd+bwd per step over rotated buffer copies, HIP
    graph replays on the fastest of 1-3 streams; per-call durations from HIP events on eager
    launches.  With `full`, also the compact hit form, the per-event launches and the steps either
    side of the chain."""
    import numpy as np
    import torch

    import synth
    import paper_2002_11529_amd as utc

    dev = torch.device("cuda:0")
    b = synth.generate(workload, n_events=args.events if workload == args.workload else None,
                       with_truth=False)
    E, S = b.n_events, b.detector.n_sectors
    NB = E * 4 * S
    geom = utc.Geometry(b.detector, dev)
    params = utc.compass_params(b.params)
    L = utc.library()
    print(f"[bench] {workload}: {E} events, {b.n_tracks} tracks, {b.n_words} words", file=sys.stderr,
          flush=True)

    NS_CHOICES = (1, 2, 3) if args.streams <= 0 else (args.streams,)
    LCM = int(np.lcm.reduce(NS_CHOICES))
    R = -(-max(1, args.rotate, LCM) // LCM) * LCM   # a multiple of every stream count tried
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
        # workspaces per copy: steps on different streams may run at the same time
        ws = dict(dec=torch.empty(L.ut_decode_workspace_bytes(E, S), dtype=torch.uint8, device=dev),
                  find=torch.empty(max(256, L.compass_find_workspace_bytes(E, b.n_tracks)),
                                   dtype=torch.uint8, device=dev),
                  fg=torch.empty(L.compass_fit_grad_workspace_bytes(S), dtype=torch.uint8, device=dev))
        copies.append(dict(words=words, boff=boff, vel=vel, vo=vo, hits=hits, res=res, fg=fg, ws=ws))
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    offsets = torch.zeros(4 * S, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_autotune:
        c0 = copies[0]
        tuned = utc.autotune(geom, params, E, c0["words"], c0["boff"], *c0["vel"], c0["vo"], reps=5)
    lau_dec = tuned["decode"] if tuned else None
    lau_find = tuned["find"] if tuned else None

    def step(c, ev=None, compact=False, lf=lau_find):
        stream = torch.cuda.current_stream()
        # the compact form passes no z / y_begin / y_end: the decoder skips those stores and the
        # search takes the detector's y range for every strip
        hits = {k: c["hits"][k] for k in ("hit_offsets", "lhcbid", "u", "weight")} if compact else c["hits"]
        if ev is not None:
            ev[0].record(stream)
        utc.ut_decode(geom, c["words"], c["boff"], E, hit_capacity=b.n_words, error_flags=flags,
                      out=hits, workspace=c["ws"]["dec"], launch=lau_dec)
        if ev is not None:
            ev[1].record(stream)
        utc.compass_find(geom, params, E, hits, *c["vel"], c["vo"], error_flags=flags,
                         out=c["res"], workspace=c["ws"]["find"], launch=lf)
        if ev is not None:
            ev[2].record(stream)
        utc.compass_fit_grad(geom, c["res"]["hit_idx"], hits["u"], hits["weight"],
                             hits["lhcbid"], *c["vel"], c["res"]["qop"], offsets,
                             out=c["fg"], workspace=c["ws"]["fg"])
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

    # the search's launch shapes tried with the stream counts: the tuned one (timed on one stream)
    # and, when that is a persistent grid, one workgroup per event, whose uneven tails leave room
    # for the steps on other streams
    find_choices = [lau_find]
    if lau_find and 0 < lau_find["grid"] < E:
        find_choices.append({"block": 256, "grid": 0, "tile": lau_find.get("tile", 0)})

    # the step captured once per buffer copy (and search shape) in a HIP graph, replayed
    graph_sets = None
    if not args.no_graph:
        graph_sets = []
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for lf in find_choices:
                gs = []
                for c in copies:
                    gph = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(gph, stream=side):
                        step(c, lf=lf)
                    gs.append(gph)
                graph_sets.append(gs)
        torch.cuda.current_stream().wait_stream(side)
        stream = torch.cuda.current_stream()
        for gs in graph_sets:
            for i in range(args.warmup):
                gs[i % R].replay()
        torch.cuda.synchronize()
    graphs = graph_sets[0] if graph_sets else None

    # K whole steps, bracketed by synchronisation; step i runs on stream i % ns
    side_streams = [torch.cuda.Stream() for _ in range(max(NS_CHOICES) - 1)]

    def run_steps(ns, k, gi=0):
        streams = [stream] + side_streams[:ns - 1]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record(stream)
        for st in streams[1:]:
            st.wait_stream(stream)
        for i in range(k):
            with torch.cuda.stream(streams[i % ns]):
                if graph_sets is not None:
                    graph_sets[gi][i % R].replay()
                else:
                    step(copies[i % R], lf=find_choices[gi])
        for st in streams[1:]:
            stream.wait_stream(st)
        t_end.record(stream)
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end), time.perf_counter() - wall0

    # the stream count (and search shape): the fastest of the candidates over short bursts (twice
    # each, best kept)
    stream_trials = None
    NS, GI = NS_CHOICES[0], 0
    if len(NS_CHOICES) > 1 or len(find_choices) > 1:
        kt = max(2 * LCM, min(K // 2, 60))
        trials = {(ns, gi): min(run_steps(ns, kt, gi)[0] for _ in range(2)) / kt
                  for gi in range(len(find_choices)) for ns in NS_CHOICES}
        NS, GI = min(trials, key=trials.get)
        name = (lambda ns, gi: str(ns)) if len(find_choices) == 1 else \
               (lambda ns, gi: f"{ns} streams, search {launch_tag(find_choices[gi], E)}")
        stream_trials = {name(ns, gi): round(ms, 5) for (ns, gi), ms in trials.items()}

    # the streams' first use costs milliseconds once: a warm-up pass on the chosen streams (the
    # trials above already made one), then the timed region
    if stream_trials is None:
        run_steps(NS, max(2 * R, args.warmup))
    ms_total, wall = run_steps(NS, K, GI)
    ms_per_step = ms_total / K
    if int(flags.item()) != 0:
        raise RuntimeError(f"device error flags {int(flags.item())}")

    # the same step on the compact hit form, timed the same way
    compact = None
    if full and not args.no_compact:
        gc = None
        if graphs is not None:
            gc = []
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for c in copies:
                    gph = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(gph, stream=side):
                        step(c, compact=True)
                    gc.append(gph)
            torch.cuda.current_stream().wait_stream(side)
        run = (lambda i: gc[i % R].replay()) if gc is not None else (lambda i: step(copies[i % R], compact=True))
        for i in range(args.warmup):
            run(i)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for i in range(K):
            run(i)
        c1.record(stream)
        torch.cuda.synchronize()
        if int(flags.item()) != 0:
            raise RuntimeError(f"device error flags {int(flags.item())}")
        cms = c0.elapsed_time(c1) / K
        compact = {"events_per_s": round(E / (cms * 1e-3), 1), "ms_per_step": round(cms, 5),
                   "what": "the same step on one stream with the decoder writing lhcbid/u/weight only "
                           "(12 B per hit) and the search taking the detector's y range for every strip"}
        gc = None

    # the same decode + Compass work launched one event at a time (eager), for comparison
    per_event = None
    if full and not args.no_per_event:
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
        batched_ms = float(call_ms[0] + call_ms[1])
        per_event = {"events_per_s": round(E / (pe_ms * 1e-3), 1), "ms": round(pe_ms, 3),
                     "batched_decode_compass_events_per_s": round(E / (batched_ms * 1e-3), 1),
                     "what": "ut_decode + compass_find, one event per call, eager launches, against "
                             "the same two calls over the whole batch (eager, one stream)"}
        hits2 = res2 = scratch = None

    # algorithmic bytes (each input read once, each output written once)
    Nw, Nh, Nt = b.n_words, n_valid, b.n_tracks
    bytes_decode = 2 * Nw + 4 * (NB + 1) + 4 * (NB + 1) + 24 * Nh
    bytes_find = 16 * Nt + 4 * (E + 1) + 28 * Nt
    fg_hits = int((copies[0]["res"]["hit_idx"] >= 0).sum().item())
    bytes_fg = Nt * (16 + 16 + 4 + 8) + fg_hits * 12 + 2 * 4 * (4 * S)
    bytes_step = 2 * Nw + 8 * NB + 24 * Nh + 44 * Nt
    names = ["ut_decode", "compass_find", "compass_fit_grad"]
    per_call_bytes = dict(zip(names, [bytes_decode, bytes_find, bytes_fg]))
    calls = {n: float(m) for n, m in zip(names, call_ms)}
    dom = names[int(np.argmax(call_ms))]
    shape_tags = {"k_decode": launch_tag(lau_dec, 4 * E, (lau_dec or {}).get("block", 64) // 64),
                  "k_compass": launch_tag(lau_find, E)}
    select = bench_select(args, b, geom, copies[0], E, S) if full else None
    timing = "hip graph replay" if graph_sets is not None else "eager launches"
    copies = graph_sets = graphs = None
    return {
        "batch": b, "E": E, "S": S, "Nt": Nt,
        "workload": f"{workload}: {E} events, {S} sectors/layer, {Nt} VELO tracks, {Nh} hits, "
                    f"{Nw} raw words",
        "value": E / (ms_per_step * 1e-3), "ms_per_step": ms_per_step, "wall_s": wall,
        "rotated_copies": R, "streams": NS, "search_launch_timed": find_choices[GI],
        "stream_trials": stream_trials, "calls_ms": calls, "dominant": dom,
        "per_call_GBps": {n: per_call_bytes[n] / (calls[n] * 1e-3) / 1e9 for n in names},
        "step_GBps": bytes_step / (ms_per_step * 1e-3) / 1e9,
        "shape_tags": shape_tags,
        "timing": timing,
        "launch": {"decode": lau_dec, "find": lau_find, "source": "autotuner" if tuned else "defaults",
                   "shape_tags": shape_tags},
        "per_event": per_event, "compact": compact, "found_fraction": n_found / max(Nt, 1),
        "select": select,
    }


def bench_select(args, b, geom, c, E, S):
    """The steps either side of the chain on the benchmark batch: the global event cut (limit at
    the 90th percentile of the raw words per event) and the consolidation of the found tracks."""
    import numpy as np
    import torch

    import paper_2002_11529_amd as utc

    per_event = np.diff(b.bank_offsets[::4 * S].astype(np.int64))
    limit = int(np.percentile(per_event, 90))
    L = utc.library()
    ws_cut = torch.empty(L.ut_global_event_cut_workspace_bytes(E), dtype=torch.uint8, device=c["words"].device)
    cut = utc.ut_global_event_cut(geom, E, c["words"], c["boff"], *c["vel"], c["vo"], limit, workspace=ws_cut)
    ws_cons = torch.empty(L.compass_consolidate_workspace_bytes(b.n_tracks), dtype=torch.uint8,
                          device=c["words"].device)
    cons = utc.compass_consolidate(E, c["vo"], c["res"], workspace=ws_cons)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_cut = timed(lambda: utc.ut_global_event_cut(geom, E, c["words"], c["boff"], *c["vel"], c["vo"], limit,
                                                   out=cut, workspace=ws_cut))
    ms_cons = timed(lambda: utc.compass_consolidate(E, c["vo"], c["res"], out=cons, workspace=ws_cons))
    kept = int(cut["n_kept"].item())
    kw = int(cut["bank_offsets"][-1].item())
    kt = int(cut["velo_offsets"][-1].item())
    nf = int(cons["n_found"].item())
    nb = E * 4 * S
    bytes_cut = 2 * (2 * kw + 16 * kt) + 2 * 4 * (nb + 1) + 2 * 4 * (E + 1) + E
    bytes_cons = 4 * b.n_tracks + nf * (24 + 32) + 4 * (E + 1) * 2
    return {"event_cut": {"ms": round(ms_cut, 5), "max_words": limit, "kept_events": kept,
                          "algorithmic_GBps": round(bytes_cut / (ms_cut * 1e-3) / 1e9, 1)},
            "consolidation": {"ms": round(ms_cons, 5), "found_tracks": nf,
                              "algorithmic_GBps": round(bytes_cons / (ms_cons * 1e-3) / 1e9, 1)}}


def sweep(args):
    """compass_find over the realistic workload for 1, 3 and 5 sectors and 1 to 16 hit candidates
    per window (the configurations of the paper's efficiency table and throughput figure)."""
    import numpy as np
    import torch

    import synth
    import paper_2002_11529_amd as utc
    from synth.efficiency import efficiency

    dev = torch.device("cuda:0")
    b = synth.generate(args.workload, n_events=args.events, with_truth=True)
    geom = utc.Geometry(b.detector, dev)
    words = torch.from_numpy(b.words.view(np.int16).copy()).to(dev)
    boff = torch.from_numpy(b.bank_offsets.view(np.int32).copy()).to(dev)
    vel = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (b.velo_x, b.velo_y, b.velo_tx, b.velo_ty)]
    vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(dev)
    hits = utc.ut_decode(geom, words, boff, b.n_events)
    configs = [(v, ns, m) for v in ("exhaustive", "paper") for ns in (1, 3, 5) for m in (1, 2, 4, 8, 16)]
    for variant, ns, m in configs:
        # the paper's search: windows of m hits and a budget of m tracklets
        p = synth.make_compass_params(p_min_mev=b.params.p_min, max_hits=m, n_sectors_search=ns,
                                      max_tracklets=m if variant == "paper" else 0)
        res = utc.compass_find(geom, p, b.n_events, hits, *vel, vo)
        for _ in range(args.warmup):
            utc.compass_find(geom, p, b.n_events, hits, *vel, vo, out=res)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            utc.compass_find(geom, p, b.n_events, hits, *vel, vo, out=res)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        eff = efficiency(b, res["hit_idx"].cpu().numpy(), res["nhits"].cpu().numpy())
        print(json.dumps({"workload": args.workload, "search": variant, "sectors": ns, "candidates": m,
                          "compass_find_ms": round(ms, 5),
                          "events_per_s": round(b.n_events / (ms * 1e-3), 1),
                          **{k: round(v, 5) if isinstance(v, float) else v for k, v in eff.items()}}),
              flush=True)


def copy_calibration():
    """A plain copy of known size, for scaling the HBM byte counters (FETCH_SIZE, WRITE_SIZE)."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n, "bytes_written": n, "copies": 5}), flush=True)


def valu_issue(kernel, workload, ms, launch=None):
    """The kernel's measured vector-instruction rate against the VALU issue ceiling, the bound the
    search and decode kernels actually run into (None without a current counter summary)."""
    n = measured_valu(kernel, workload, launch)
    if n is None:
        return None
    rate = n / (ms * 1e-3)
    return {"instr_per_launch": n, "achieved_instr_per_s": round(rate, -6),
            "peak_instr_per_s": VALU_ISSUE_PEAK, "frac": round(rate / VALU_ISSUE_PEAK, 4)}


def copy_bandwidth(reps=10):
    """Measured streaming bandwidth of the card: a 1 GiB device-to-device copy (read + write bytes
    per second), median of `reps` copies timed with HIP events."""
    import numpy as np
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n / (float(np.median(ms)) * 1e-3) / 1e9


def bench_fitgrad(args, dev):
    """Fit-chi2 forward + backward over the frozen tracks of the differentiation workload (21000
    events, about 1.05e6 tracks with 3 or 4 hits), against the same calls launched per event."""
    import numpy as np
    import torch

    import synth
    import paper_2002_11529_amd as utc

    b = synth.generate("fitgrad", with_truth=False)
    S = b.detector.n_sectors
    geom = utc.Geometry(b.detector, dev)
    words = torch.from_numpy(b.words.view(np.int16).copy()).to(dev)
    boff = torch.from_numpy(b.bank_offsets.view(np.int32).copy()).to(dev)
    vel = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (b.velo_x, b.velo_y, b.velo_tx, b.velo_ty)]
    vo = torch.from_numpy(b.velo_offsets.view(np.int32).copy()).to(dev)
    hits = utc.ut_decode(geom, words, boff, b.n_events)
    res = utc.compass_find(geom, b.params, b.n_events, hits, *vel, vo)
    keep = res["nhits"] >= 3
    idx = res["hit_idx"][keep].contiguous()
    st = [v[keep].contiguous() for v in vel]
    qop = res["qop"][keep].contiguous()
    off = torch.zeros(4 * S, dtype=torch.float32, device=dev)
    n = int(qop.shape[0])
    ws = torch.empty(utc.library().compass_fit_grad_workspace_bytes(S), dtype=torch.uint8, device=dev)
    # copies of every input and output used in turn, so that one call's working set (~95 MB) is not
    # still in the 256 MB Infinity Cache when the next call with the same copy starts
    R = max(3, args.rotate)
    copies = []
    for _ in range(R):
        o = dict(chi2_total=torch.empty(1, dtype=torch.float64, device=dev),
                 chi2_track=torch.empty(n, dtype=torch.float32, device=dev),
                 grad_qop=torch.empty(n, dtype=torch.float32, device=dev),
                 grad_offsets=torch.empty(4 * S, dtype=torch.float32, device=dev))
        copies.append(dict(idx=idx.clone(), st=[v.clone() for v in st], qop=qop.clone(),
                           u=hits["u"].clone(), w=hits["weight"].clone(), id=hits["lhcbid"].clone(),
                           off=off.clone(), out=o,
                           fwd=dict(chi2_total=o["chi2_total"], chi2_track=o["chi2_track"])))

    def call(c, grad):
        utc.compass_fit_grad(geom, c["idx"], c["u"], c["w"], c["id"], *c["st"], c["qop"], c["off"],
                             want_grad=grad, out=c["out"] if grad else c["fwd"], workspace=ws)

    def timed(fn, reps):
        for i in range(args.warmup):
            fn(i)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for i in range(reps):
            fn(i)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_fb = timed(lambda i: call(copies[i % R], True), args.steps)
    ms_f = timed(lambda i: call(copies[i % R], False), args.steps)
    # the same fits on the hits frozen once in track-major form (40 B per track, no gathers)
    for c in copies:
        c["fz"] = utc.compass_fit_freeze(geom, c["idx"], c["u"], c["w"], c["id"])
    ms_freeze = timed(lambda i: utc.compass_fit_freeze(geom, copies[i % R]["idx"], copies[i % R]["u"],
                                                       copies[i % R]["w"], copies[i % R]["id"],
                                                       out=copies[i % R]["fz"]), args.steps)
    ms_fz = timed(lambda i: utc.compass_fit_grad_frozen(geom, copies[i % R]["fz"], *copies[i % R]["st"],
                                                        copies[i % R]["qop"], copies[i % R]["off"],
                                                        out=copies[i % R]["out"], workspace=ws),
                  args.steps)
    out = copies[0]["out"]
    # the same work, one call per event
    ev_of_track = np.repeat(np.arange(b.n_events), np.diff(b.velo_offsets.astype(np.int64)))
    kept_per_event = np.bincount(ev_of_track[keep.cpu().numpy()], minlength=b.n_events)
    ko = np.zeros(b.n_events + 1, dtype=np.int64)
    np.cumsum(kept_per_event, out=ko[1:])
    rows = [(int(ko[e]), int(ko[e + 1])) for e in range(b.n_events) if ko[e + 1] > ko[e]]

    def per_event():
        for t0, t1 in rows:
            o = dict(chi2_total=out["chi2_total"], chi2_track=out["chi2_track"][t0:t1],
                     grad_qop=out["grad_qop"][t0:t1], grad_offsets=out["grad_offsets"])
            utc.compass_fit_grad(geom, idx[t0:t1], hits["u"], hits["weight"], hits["lhcbid"],
                                 *(v[t0:t1] for v in st), qop[t0:t1], off, out=o, workspace=ws)

    ms_pe = timed(lambda i: per_event(), 1) if not args.no_per_event else None
    n_hits = int((idx >= 0).sum().item())
    bytes_fb = n * (16 + 16 + 4 + 8) + n_hits * 12 + 2 * 4 * (4 * S)
    return {"workload": f"fitgrad: {b.n_events} events, {n} frozen tracks, {n_hits} hits, {S} sectors/layer",
            "fwd_bwd_tracks_per_s": round(n / (ms_fb * 1e-3), 1), "fwd_bwd_ms": round(ms_fb, 5),
            "fwd_only_tracks_per_s": round(n / (ms_f * 1e-3), 1), "fwd_only_ms": round(ms_f, 5),
            "fwd_bwd_algorithmic_GBps": round(bytes_fb / (ms_fb * 1e-3) / 1e9, 1),
            "rotated_copies": R,
            "frozen_layout": {"fwd_bwd_tracks_per_s": round(n / (ms_fz * 1e-3), 1),
                              "fwd_bwd_ms": round(ms_fz, 5),
                              "algorithmic_GBps": round((n * (16 + 4 + 40 + 8) + 2 * 4 * (4 * S)) /
                                                        (ms_fz * 1e-3) / 1e9, 1),
                              "freeze_ms": round(ms_freeze, 5),
                              "what": "compass_fit_grad_frozen on u, weight and sector gathered once per "
                                      "track by compass_fit_freeze (same results)"},
            "per_event_launch_tracks_per_s": round(n / (ms_pe * 1e-3), 1) if ms_pe else None,
            "per_event_launch_ms": round(ms_pe, 3) if ms_pe else None,
            "per_event_what": "compass_fit_grad fwd+bwd, one call per event (the offset gradient of "
                              "each call overwrites the last; no cross-event sum)"}


def host_cpu_info():
    """What the host offers this process: logical CPUs, the affinity set, the cgroup CPU quota
    (cpu.max, in CPUs) and the CPU model."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cgroup_cpus": None,
            "model": None}
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            info["cgroup_cpus"] = round(int(q) / int(per), 2)
    except (OSError, ValueError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


# CPUs a one-GPU job may keep busy on the GPU host (its share of the host), whatever the host
# reports as online
HOST_CPU_SHARE = 16


def cpu_baseline(b, seconds, n_events=2000):
    """The oracle (decode + Compass + fit-chi2 fwd+bwd) on a bounded sample of the same workload:
    the first `n_events` events.  Timed on every CPU of this process's host share (events are
    independent, so the sample is split into one slice per thread; the oracle's C calls release
    the interpreter lock), and on one thread.  Events/s of the sample stand for the whole batch."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth

    def one_pass(sub):
        d = oracle.decode(sub.detector, sub.words, sub.bank_offsets, sub.n_events)
        c = oracle.compass(sub.detector, sub.params, sub.n_events, d, sub.velo_x, sub.velo_y,
                           sub.velo_tx, sub.velo_ty, sub.velo_offsets)
        oracle.fit_grad(sub.detector, c["hit_idx"], d["u"], d["weight"], d["lhcbid"], sub.velo_x,
                        sub.velo_y, sub.velo_tx, sub.velo_ty, c["qop"],
                        np.zeros(4 * sub.detector.n_sectors, np.float32))

    info = host_cpu_info()
    m = min(b.n_events, n_events)
    sub = synth.take_events(b, np.arange(m)) if m < b.n_events else b
    share = [info["affinity"], HOST_CPU_SHARE]
    if info["cgroup_cpus"]:
        share.append(int(info["cgroup_cpus"]))
    cores = max(1, min(*share, sub.n_events))
    cuts = np.linspace(0, sub.n_events, cores + 1).astype(np.int64)
    slices = [synth.take_events(sub, np.arange(cuts[i], cuts[i + 1])) for i in range(cores)]
    budget = seconds / 2

    def worker(sl):
        n, t1 = 0, time.perf_counter()
        while True:
            one_pass(sl)
            n += sl.n_events
            if time.perf_counter() - t1 >= budget:
                return n

    t1 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        done = sum(ex.map(worker, slices))
    t_all = time.perf_counter() - t1
    value = done / t_all

    reps, t0 = 0, time.perf_counter()
    while True:
        one_pass(sub)
        reps += 1
        t_one = time.perf_counter() - t0
        if t_one >= budget:
            break
    one = reps * sub.n_events / t_one
    return {"value": round(value, 1), "unit": "events/s", "cores": cores, "kind": "oracle",
            "sample": f"the first {sub.n_events} of the {b.n_events} events (decode + Compass + "
                      f"fit-chi2 fwd+bwd), split over {cores} threads, each repeating its slice for "
                      f"{budget:.0f} s ({t_all:.1f} s wall); the rate stands for the whole batch "
                      f"({b.n_events / value:.1f} s extrapolated)",
            "host": info, "host_share_cpus": HOST_CPU_SHARE,
            "single_thread": {"value": round(one, 1), "unit": "events/s", "cores": 1,
                              "sample": f"{reps} passes over the same {sub.n_events} events, "
                                        f"{t_one:.1f} s"}}


if __name__ == "__main__":
    main()
