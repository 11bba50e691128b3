"""The oracle on the hand-worked fixtures of tests/golden/: the search order of the paper's variant
(central sector first, anchor pairs A-major, closest completion hit to the pair-slope line, first in
walk order on a tie), the weight and NaN rules of the selection, and the acceptance boundary at the
first and last layer (Sections V-A, V-B).  Each fixture states its derivation."""
import numpy as np
import pytest

import oracle
import synth
from tests.golden_search import build_event, load_acceptance_tracks, load_search_cases

CASES = load_search_cases()


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_search_fixture(case):
    det, par, hits, st, expect = build_event(case)
    c = oracle.compass(det, par, 1, hits, *st, np.array([0, 1], np.uint32), with_windows=True)
    assert c["active"][0] == 1
    assert list(c["hit_idx"][0]) == expect
    assert c["nhits"][0] == sum(i >= 0 for i in expect)


def test_fixture_cases_present():
    names = {c["name"] for c in CASES}
    assert {"central_first_budget_1", "central_first_budget_2", "completion_tie_walk_order",
            "completion_closest_to_pair_slope", "pair_order_a_major", "negative_weight_unusable",
            "nan_weight_unusable", "nan_chi2_ranks_last", "nan_chi2_tie_by_index"} <= names


def test_nan_chi2_outputs():
    """A selected candidate whose hits all weigh 0 reports q/p and chi2 as NaN."""
    case = next(c for c in CASES if c["name"] == "nan_chi2_tie_by_index")
    det, par, hits, st, expect = build_event(case)
    c = oracle.compass(det, par, 1, hits, *st, np.array([0, 1], np.uint32))
    assert np.isnan(c["qop"][0]) and np.isnan(c["chi2"][0]) and c["nhits"][0] == 4


def test_acceptance_fixture():
    states, active = load_acceptance_tracks()
    det = synth.make_detector(32)
    par = synth.make_compass_params()
    hits = dict(hit_offsets=np.zeros(4 * 32 + 1, np.uint32), u=np.zeros(1, np.float32),
                weight=np.zeros(1, np.float32), y_begin=np.zeros(1, np.float32),
                y_end=np.zeros(1, np.float32))
    n = len(active)
    c = oracle.compass(det, par, 1, hits, states[:, 0], states[:, 1], states[:, 2], states[:, 3],
                       np.array([0, n], np.uint32), with_windows=True)
    assert list(c["active"]) == list(active)
    assert np.all(c["win_first"][active == 0] == -1)
