"""Pins of the bipartite K-best oracle (oracle/bipartite_oracle.c) against an
independent brute force over every vertex mapping (tests/_pins.py): the popped
assignment costs are the K smallest over all mappings in non-decreasing order,
each popped mapping is distinct and has the stated cost, the distance is the
least induced cost among them, K covering every mapping gives the exact GED,
and the bound never grows with K."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import Graph
from tests import _pins

UNIT = synth.UNIT_COSTS
PAPER = synth.PAPER_COSTS
HIGH = (4, 12, 12, 1, 10, 10)
NONMETRIC = (3, 2, 5, 9, 1, 2)      # esub > edel + eins
ODD = (3, 1, 2, 5, 1, 3)


def tiny_pairs(seed, count, n_max, p, nvl, nel):
    gs = [synth.random_small_graph(seed, k, n_max, p, nvl, nel) for k in range(2 * count)]
    return [(gs[2 * k], gs[2 * k + 1]) for k in range(count)]


def brute(g1, g2, c):
    inc1, inc2 = _pins.incident_labels(g1), _pins.incident_labels(g2)
    maps = list(_pins.all_mappings(int(g1.n), int(g2.n)))
    bc = [_pins.bipartite_cost(g1, g2, c, m, inc1, inc2) for m in maps]
    ic = [_pins.qap_cost(g1, g2, c, _pins.perm_from_map(m, int(g1.n), int(g2.n))) for m in maps]
    return maps, np.asarray(bc, np.int64), np.asarray(ic, np.int64)


@pytest.mark.parametrize("costs", [UNIT, PAPER, HIGH, NONMETRIC, ODD])
def test_popped_costs_are_the_k_smallest(costs):
    for g1, g2 in tiny_pairs(11, 6, 4, 0.5, 2, 3):
        maps, bc, ic = brute(g1, g2, costs)
        total = len(maps)
        for K in (1, 2, 5, 17, total, total + 3):
            d, mp, solves, pc, pm = oracle.bipartite(g1, g2, costs, K, trace=True)
            k = min(K, total)
            assert len(pc) == k
            np.testing.assert_array_equal(pc, np.sort(bc)[:k])
            seen = set()
            for q in range(k):
                key = tuple(int(x) for x in pm[q])
                assert key not in seen
                seen.add(key)
                assert _pins.bipartite_cost(g1, g2, costs, key) == pc[q]
            ind = [_pins.qap_cost(g1, g2, costs, _pins.perm_from_map(pm[q], int(g1.n), int(g2.n)))
                   for q in range(k)]
            first = int(np.argmin(ind))
            assert d == ind[first]
            np.testing.assert_array_equal(mp, pm[first])
            assert 1 <= solves <= 1 + min(K - 1, k) * int(g1.n)


@pytest.mark.parametrize("costs", [UNIT, PAPER, NONMETRIC])
def test_all_mappings_give_exact(costs):
    for g1, g2 in tiny_pairs(13, 5, 4, 0.6, 2, 2):
        maps, bc, ic = brute(g1, g2, costs)
        d, mp, _ = oracle.bipartite(g1, g2, costs, len(maps))
        assert d == ic.min() == _pins.qap_exact(g1, g2, costs)


def test_bound_never_grows_with_k():
    for g1, g2 in tiny_pairs(17, 8, 7, 0.4, 3, 2):
        prev = None
        for K in range(1, 40):
            d, _, _ = oracle.bipartite(g1, g2, PAPER, K)
            ex = None
            if prev is not None:
                assert d <= prev
            prev = d
        assert prev >= oracle.exact(g1, g2, PAPER)[0]


def test_local_edge_cost_closed_form_cases():
    """Hand cases of the incident-edge assignment that the closed form in the
    oracle must reproduce: label multisets, more and fewer edges, non-metric."""
    c = (0, 0, 0, 5, 2, 1)          # esub 5 > edel + eins = 3: relabel by delete + insert
    assert _pins.edge_assignment_cost([1, 1, 2], [1, 3], c) == 0 * 1 + 3 + 2
    c2 = (0, 0, 0, 1, 2, 1)
    assert _pins.edge_assignment_cost([1, 1, 2], [1, 3], c2) == 1 + 2
    assert _pins.edge_assignment_cost([], [4, 4], c2) == 2
    # one pair through the oracle: a star against a path, unit costs
    g1 = Graph(n=3, vlabel=np.zeros(3, np.int32), eu=np.array([0, 0], np.int32), ev=np.array([1, 2], np.int32))
    g2 = Graph(n=3, vlabel=np.zeros(3, np.int32), eu=np.array([0, 1], np.int32), ev=np.array([1, 2], np.int32))
    d, mp, s, pc, pm = oracle.bipartite(g1, g2, UNIT, 1, trace=True)
    assert pc[0] == 0 and d == 0      # centre to centre: identical incident edges


def test_empty_graphs():
    e = Graph(n=0, vlabel=np.zeros(0, np.int32), eu=np.zeros(0, np.int32), ev=np.zeros(0, np.int32))
    g = synth.random_small_graph(19, 0, 6, 0.5, 2, 1)
    g = g if g.n > 0 else synth.random_small_graph(19, 1, 6, 0.5, 2, 1)
    c = PAPER
    d, mp, s = oracle.bipartite(e, g, c, 5)
    assert d == c[2] * g.n + c[5] * len(g.eu) and s == 1 and mp.size == 0
    d, mp, s = oracle.bipartite(g, e, c, 5)
    assert d == c[1] * g.n + c[4] * len(g.eu) and (mp == -1).all()
    d, mp, s = oracle.bipartite(e, e, c, 1)
    assert d == 0


def test_identical_graph_reaches_zero():
    """GED(G, G) = 0 once K covers the mappings of zero assignment cost (vertex
    pairs with equal labels and incident labels tie at zero; K = 1 need not
    find the identity)."""
    for g, _ in tiny_pairs(23, 5, 5, 0.5, 3, 2):
        maps, bc, ic = brute(g, g, UNIT)
        zero = int((bc == 0).sum())
        d, _, _ = oracle.bipartite(g, g, UNIT, max(zero, 1))
        assert d == 0


def test_pairs_entry_matches_single():
    gs = [synth.random_small_graph(29, k, 9, 0.4, 3, 2) for k in range(10)]
    graphs = synth.GraphSet.from_graphs(gs)
    pairs = np.array([[0, 1], [2, 3], [4, 4], [5, 9], [9, 5]], np.int64)
    d, m, off, s = oracle.bipartite_pairs(graphs, pairs, HIGH, 12)
    for q, (a, b) in enumerate(pairs):
        d1, m1, s1 = oracle.bipartite(gs[a], gs[b], HIGH, 12)
        assert d[q] == d1 and s[q] == s1
        np.testing.assert_array_equal(m[off[q]:off[q] + gs[a].n], m1)
