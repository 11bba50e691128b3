"""Plain definitions of the steps on either side of the UT chain (Section VI, "UT decoding and
tracking performance"): the global event cut before decoding and the consolidation of the found
upstream tracks after the tracking.

TEST INFRASTRUCTURE ONLY (like the rest of this package): written event by event and track by
track from the definitions, with no blocking or reordering.
"""
from __future__ import annotations

import numpy as np

N_LAYERS = 4


def global_event_cut(n_sectors, n_events, words, bank_offsets, vx, vy, vtx, vty, velo_offsets,
                     max_words):
    """An event is kept when its raw banks hold at most max_words words (padding included) and its
    bank offsets do not decrease from its first to its last bank; the result has the same events,
    the rejected ones empty (no words, every bank empty, no VELO tracks)."""
    bpe = N_LAYERS * n_sectors
    bo = np.asarray(bank_offsets, np.int64)
    vo = np.asarray(velo_offsets, np.int64)
    out_words, out_bo, keep = [], [0], []
    out_state = [[], [], [], []]
    out_vo = [0]
    for e in range(n_events):
        a, b = bo[e * bpe], bo[(e + 1) * bpe]
        ok = b >= a and b - a <= max_words
        keep.append(1 if ok else 0)
        base = out_bo[-1]
        for i in range(e * bpe + 1, (e + 1) * bpe + 1):
            out_bo.append(base + (bo[i] - a) if ok else base)
        if ok:
            out_words.append(np.asarray(words[a:b], np.uint16))
            for k, arr in enumerate((vx, vy, vtx, vty)):
                out_state[k].append(np.asarray(arr[vo[e]:vo[e + 1]], np.float32))
            out_vo.append(out_vo[-1] + (vo[e + 1] - vo[e]))
        else:
            out_vo.append(out_vo[-1])

    def cat(parts, dtype):
        return np.concatenate(parts).astype(dtype) if parts else np.zeros(0, dtype)

    return dict(words=cat(out_words, np.uint16), bank_offsets=np.array(out_bo, np.uint32),
                vx=cat(out_state[0], np.float32), vy=cat(out_state[1], np.float32),
                vtx=cat(out_state[2], np.float32), vty=cat(out_state[3], np.float32),
                velo_offsets=np.array(out_vo, np.uint32), keep=np.array(keep, np.uint8),
                n_kept=int(sum(keep)))


def consolidate(n_events, velo_offsets, nhits, hit_idx, qop, chi2):
    """The tracks with nhits > 0, in VELO order, and offsets[e] = number of them in events before e."""
    vo = np.asarray(velo_offsets, np.int64)
    velo, idx, q, c, nh, offsets = [], [], [], [], [], [0]
    for e in range(n_events):
        for t in range(vo[e], vo[e + 1]):
            if nhits[t] > 0:
                velo.append(t)
                idx.append(np.asarray(hit_idx[t], np.int32))
                q.append(qop[t])
                c.append(chi2[t])
                nh.append(nhits[t])
        offsets.append(len(velo))
    return dict(offsets=np.array(offsets, np.uint32), velo=np.array(velo, np.int32),
                hit_idx=np.array(idx, np.int32).reshape(-1, 4), qop=np.array(q, np.float32),
                chi2=np.array(c, np.float32), nhits=np.array(nh, np.int32), n_found=len(velo))
