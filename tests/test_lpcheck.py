"""CPU tests of the parity checker itself (tests/lpcheck.py) and of the
oracle's pair-by-pair route it relies on: a GPU list that swaps tied pairs
passes; one that holds a non-candidate, a wrong score or a pair clearly below
the k-th score fails."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from lpcheck import assert_query_rows, assert_same_list

MEAS = oracle.MEASURES


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("L", [2, 5, None])
def test_pairs_matches_bruteforce(seed, L):
    """oracle.pairs on every ordered pair of a small random graph agrees with
    the candidate list of oracle.bruteforce (both orientations)."""
    g = synth.random_graph(40, 0.12, seed)
    for m in ("CN", "JC", "AA", "RA"):
        bf = oracle.bruteforce(g, L, m)
        ref = {(int(a), int(c)): (int(h), float(s)) for a, c, h, s in zip(bf["a"], bf["c"], bf["h"], bf["s"])}
        a, c = np.array(list(itertools.permutations(range(g.n), 2)), np.int32).T
        ok, h, s = oracle.pairs(g, L, m, a, c)
        for i in range(a.shape[0]):
            key = (min(a[i], c[i]), max(a[i], c[i]))
            if key in ref:
                assert ok[i] and h[i] == ref[key][0] and s[i] == ref[key][1]
            else:
                assert not ok[i]


def _star():
    return synth.from_edges(6, [(0, i) for i in range(1, 6)])


def _list(g, pairs, m, L=None):
    a = np.array([p[0] for p in pairs], np.int32)
    c = np.array([p[1] for p in pairs], np.int32)
    _, _, s = oracle.pairs(g, L, m, a, c)
    return a, c, s.astype(np.float32)


def test_tied_swap_passes():
    """K_{1,5}: all ten leaf pairs tie under AA; any four of them are a correct top 4."""
    g = _star()
    ref = oracle.predict(g, None, "AA", 4)
    got = _list(g, [(1, 2), (1, 3), (1, 4), (2, 5)], "AA")
    assert_same_list(got, ref, "AA", "tied swap", graph=g, L=None)


def test_non_candidate_fails():
    """An adjacent pair reported with the tied score is not a candidate."""
    g = _star()
    ref = oracle.predict(g, None, "AA", 4)
    a, c, s = _list(g, [(1, 2), (1, 3), (1, 4), (2, 5)], "AA")
    a[0], c[0] = 0, 1  # centre - leaf: an edge of the graph
    o = np.lexsort((c, a, -s.astype(np.float64)))
    with pytest.raises(AssertionError, match="not a candidate"):
        assert_same_list((a[o], c[o], s[o]), ref, "AA", "edge", graph=g, L=None)


def test_wrong_score_fails():
    """A real candidate outside the oracle's list whose reported score is the
    k-th score but whose true score is lower."""
    g = synth.from_edges(7, [(a, b) for a in range(3) for b in range(3, 7)])  # K_{3,4}
    ref = oracle.predict(g, None, "RA", 3)  # the three A-pairs, RA = 4/3
    a, c, s = ref["a"].copy(), ref["c"].copy(), ref["s32"].copy()
    a[2], c[2] = 3, 4  # a B-pair (RA = 3/4) reported at 4/3
    o = np.lexsort((c, a, -s.astype(np.float64)))
    with pytest.raises(AssertionError):
        assert_same_list((a[o], c[o], s[o]), ref, "RA", "wrong score", graph=g, L=None)


def test_below_kth_fails():
    """A real candidate with its own (correct) score, clearly below the k-th."""
    g = synth.from_edges(7, [(a, b) for a in range(3) for b in range(3, 7)])
    ref = oracle.predict(g, None, "AA", 3)
    a, c, s = ref["a"].copy(), ref["c"].copy(), ref["s32"].copy()
    _, _, s34 = oracle.pairs(g, None, "AA", [3], [4])
    a[2], c[2], s[2] = 3, 4, np.float32(s34[0])
    with pytest.raises(AssertionError, match="clearly below"):
        assert_same_list((a, c, s), ref, "AA", "below", graph=g, L=None)


def test_missing_graph_fails():
    """Pairs outside the oracle's list cannot pass unchecked."""
    g = _star()
    ref = oracle.predict(g, None, "AA", 4)
    got = _list(g, [(1, 2), (1, 3), (1, 4), (2, 5)], "AA")
    with pytest.raises(AssertionError, match="no graph"):
        assert_same_list(got, ref, "AA", "no graph")


def test_query_rows_checks_off_list():
    """Query rows: a tied swap passes, a neighbour of the source fails."""
    g = _star()
    src = np.array([1], np.int32)
    refq = oracle.query(g, None, "RA", src, 2)  # leaves 2..5 tie at 0.2
    c = np.array([[3, 5]], np.int32)
    s = np.full((1, 2), np.float32(0.2))
    assert_query_rows(c, s, [2], src, refq, "RA", "swap", graph=g, L=None)
    c_bad = np.array([[0, 3]], np.int32)  # 0 is the source's neighbour
    with pytest.raises(AssertionError, match="not a candidate"):
        assert_query_rows(c_bad, s, [2], src, refq, "RA", "neighbour", graph=g, L=None)
