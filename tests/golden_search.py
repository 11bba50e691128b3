"""Loaders of the hand-worked search fixtures (tests/golden/search_cases.txt and
acceptance_tracks.txt): they only turn the text into input arrays and expected hit labels."""
import os

import numpy as np

import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
N_SECTORS = 32


def load_search_cases():
    cases, cur = [], None
    for raw in open(os.path.join(HERE, "search_cases.txt")):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], hits=[], params={})
        elif tok[0] == "params":
            cur["params"] = {k: int(v) for k, v in (t.split("=") for t in tok[1:])}
        elif tok[0] == "track":
            cur["track"] = [float(v) for v in tok[1:5]]
        elif tok[0] == "hit":
            w = float(tok[5]) if len(tok) > 5 else 400.0
            cur["hits"].append(dict(label=tok[1], layer=int(tok[2]), sector=int(tok[3]),
                                    u=np.float32(tok[4]), weight=np.float32(w)))
        elif tok[0] == "expect":
            cur["expect"] = tok[1:5]
        elif tok[0] == "end":
            cases.append(cur)
            cur = None
    return cases


def build_event(case):
    """Detector, params, the hit structure of arrays (banks in (layer, sector) order, hits of a
    bank in the order listed) and the label -> global hit index map of one case."""
    det = synth.make_detector(N_SECTORS)
    par = synth.make_compass_params(**case["params"])
    S = N_SECTORS
    by_bank = {}
    for h in case["hits"]:
        by_bank.setdefault(h["layer"] * S + h["sector"], []).append(h)
    ho = np.zeros(4 * S + 1, np.uint32)
    u, w, index = [], [], {}
    for bank in range(4 * S):
        hs = by_bank.get(bank, [])
        assert all(hs[i]["u"] <= hs[i + 1]["u"] for i in range(len(hs) - 1)), "hits of a bank in ascending u"
        for h in hs:
            index[h["label"]] = len(u)
            u.append(h["u"])
            w.append(h["weight"])
        ho[bank + 1] = len(u)
    n = len(u)
    hits = dict(hit_offsets=ho, u=np.array(u, np.float32), weight=np.array(w, np.float32),
                y_begin=np.full(n, det.y_begin, np.float32), y_end=np.full(n, det.y_end, np.float32))
    x0, y0, tx, ty = (np.array([v], np.float32) for v in case["track"])
    expect = [index[lab] if lab != "-" else -1 for lab in case["expect"]]
    return det, par, hits, (x0, y0, tx, ty), expect


def load_acceptance_tracks():
    rows = []
    for raw in open(os.path.join(HERE, "acceptance_tracks.txt")):
        line = raw.split("#", 1)[0].strip()
        if line.startswith("track"):
            t = line.split()
            rows.append(([float(v) for v in t[1:5]], int(t[5])))
    states = np.array([r[0] for r in rows], np.float64)
    for col in range(4):   # every value is exact in binary32
        assert np.array_equal(states[:, col].astype(np.float32).astype(np.float64), states[:, col])
    return states.astype(np.float32), np.array([r[1] for r in rows], np.uint8)
