"""Physics-efficiency figures of found upstream tracks against the generator's truth, following the
definitions of Section III-B: a particle is reconstructible with hits in at least three of the four
layers; a found track is associated with (reconstructs) a particle when at least 70 % of its hits
come from it; efficiency = reconstructed and reconstructible particles / reconstructible particles;
clone rate = clone tracks / all found tracks and fake rate = fake tracks / all found tracks, a clone
being a track associated with a particle that an earlier track already reconstructs and a fake a
track associated with none.  Adapted to the synthetic set-up: a track's hits are its UT hits (the
VELO segment is the particle's own by construction); one output slot per VELO track, so a clone
is a second VELO track whose UT hits belong to the same particle.

Needs a batch generated with truth.  Only truth bookkeeping: no arithmetic of the method.
"""
from __future__ import annotations

import numpy as np

from .events import EventBatch, N_LAYERS


def decoded_hit_truth(batch: EventBatch) -> np.ndarray:
    """Truth id of every decoded hit, in the decoder's output order: valid words of each bank,
    ordered by word value, ties in raw order (the decoder's order), banks in raw order."""
    words = batch.words.astype(np.int64)
    valid = (words & 0xF) != 0
    nb = batch.bank_offsets.shape[0] - 1
    bank = np.repeat(np.arange(nb, dtype=np.int64), np.diff(batch.bank_offsets.astype(np.int64)))
    idx = np.nonzero(valid)[0]
    order = np.lexsort((idx, words[idx], bank[idx]))   # bank, then word value, then raw position
    return batch.truth["track"][idx[order]].astype(np.int64)


def associated(ids: np.ndarray, min_fraction: float = 0.7) -> int:
    """The particle a track with hit truth ids `ids` is associated with, or -1: the most frequent id
    when it is a particle (>= 0) and at least min_fraction of the hits carry it.  The fraction is
    compared exactly (as a ratio of integers), so 7 of 10 hits is 70 %."""
    from fractions import Fraction
    if ids.size == 0:
        return -1
    vals, counts = np.unique(ids, return_counts=True)
    k = int(np.argmax(counts))
    f = Fraction(min_fraction).limit_denominator(1000)
    if vals[k] >= 0 and int(counts[k]) * f.denominator >= f.numerator * int(ids.size):
        return int(vals[k])
    return -1


def efficiency(batch: EventBatch, hit_idx: np.ndarray, nhits: np.ndarray, min_fraction: float = 0.7):
    """Efficiency, clone rate and fake rate of the found tracks (nhits > 0) of one search.

    A found track is associated with particle P when at least min_fraction of its hits come from P
    (noise hits and hits of particles without a VELO track cannot be associated).  Efficiency: the
    reconstructible VELO particles with an associated track; clones: associated tracks beyond the
    first of their particle; fakes: found tracks associated with no particle; both rates over all
    found tracks (Section III-B)."""
    truth = decoded_hit_truth(batch)
    n = batch.n_tracks
    reconstructible = batch.n_layers_hit >= 3
    found = np.nonzero(nhits > 0)[0]
    idx = np.asarray(hit_idx, np.int64).reshape(n, N_LAYERS)
    assoc = np.full(n, -1, np.int64)   # particle associated with the track of VELO slot t
    for t in found:
        assoc[t] = associated(truth[idx[t][idx[t] >= 0]], min_fraction)
    matched = assoc[found]
    matched = matched[matched >= 0]
    particles = np.unique(matched)
    n_found = int(found.size)
    hit_particles = np.zeros(n, bool)
    hit_particles[particles] = True
    n_reco = int(reconstructible.sum())
    return {"reconstructible": n_reco,
            "efficiency": float((hit_particles & reconstructible).sum() / max(n_reco, 1)),
            "clone_rate": float((matched.size - particles.size) / max(n_found, 1)),
            "fake_rate": float((n_found - matched.size) / max(n_found, 1)),
            "found": n_found}
