"""Pins of the oracle's directed mode (edge k is the arc eu[k] -> ev[k]; each
arc one edit operation; the implied operations of Sec. 2.3 taken for both
arc directions between the edited vertex and each earlier one).

Each pin reaches the value by another route:
* hand-derived values on two- and three-vertex graphs;
* the padded-permutation form over ordered vertex pairs (tests/_pins.py),
  for every mapping and for the exact minimum;
* the K-Best search recomputed from scratch per child (tests/_pins.py);
* symmetric closure: a directed graph holding both arcs of every edge of an
  undirected graph has, for every mapping and every K, exactly the cost and
  result of the undirected search with the three edge costs doubled;
* arc reversal in both graphs changes no cost and no result;
* the search's distance is the induced cost of its mapping, and large K
  reaches the exact GED (Sec. 4.5).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import Graph
from tests import _pins

pytestmark = pytest.mark.filterwarnings("ignore")

UNIT = synth.UNIT_COSTS
PAPER = synth.PAPER_COSTS
NONMETRIC = (3, 2, 5, 9, 1, 2)
ALL_COSTS = [UNIT, PAPER, NONMETRIC, (1, 1, 1, 7, 5, 3)]


def dg(n, arcs, vl=None, el=None):
    arcs = list(arcs)
    return Graph(n, np.asarray(vl if vl is not None else [0] * n, np.int32),
                 np.asarray([a for a, _ in arcs], np.int32).reshape(-1),
                 np.asarray([b for _, b in arcs], np.int32).reshape(-1),
                 None if el is None else np.asarray(el, np.int32))


def tiny_directed(seed, k, n_max, p, nl, nel=0, n_min=0):
    return synth.directed_graph(seed, k, n_min, n_max, p, p, nl, nel)


def reversed_graph(g):
    return Graph(g.n, g.vlabel, g.ev.copy(), g.eu.copy(), None if g.elabel is None else g.elabel.copy())


def symmetric_closure(g):
    """Both arcs of every undirected edge, each with the edge's label."""
    el = None if g.elabel is None else np.concatenate([g.elabel, g.elabel])
    return Graph(g.n, g.vlabel, np.concatenate([g.eu, g.ev]).astype(np.int32),
                 np.concatenate([g.ev, g.eu]).astype(np.int32), el)


def doubled_edges(c):
    return (c[0], c[1], c[2], 2 * c[3], 2 * c[4], 2 * c[5])


# ---------------------------------------------------------------- hand values
def test_reversed_arc_maps_onto_itself():
    """g1: 0 -> 1, g2: 1 -> 0 (same vertex labels): swapping the vertices costs 0;
    the identity deletes one arc and inserts the other."""
    g1, g2 = dg(2, [(0, 1)]), dg(2, [(1, 0)])
    for c in ALL_COSTS:
        assert oracle.induced_cost(g1, g2, c, [1, 0], directed=True) == 0
        assert oracle.induced_cost(g1, g2, c, [0, 1], directed=True) == c[4] + c[5]
        assert oracle.exact(g1, g2, c, directed=True)[0] == 0
        # undirected, both graphs are the same edge: identity costs 0
        assert oracle.induced_cost(g1, g2, c, [0, 1]) == 0


def test_two_cycle_against_one_arc():
    """g1 has both arcs 0 <-> 1, g2 only 0 -> 1: one arc deleted whichever way round,
    unless deleting vertices is cheaper."""
    g1, g2 = dg(2, [(0, 1), (1, 0)]), dg(2, [(0, 1)])
    for c in ALL_COSTS:
        assert oracle.induced_cost(g1, g2, c, [0, 1], directed=True) == c[4]
        assert oracle.induced_cost(g1, g2, c, [1, 0], directed=True) == c[4]
        assert oracle.induced_cost(g1, g2, c, [-1, -1], directed=True) == 2 * c[1] + 2 * c[4] + 2 * c[2] + c[5]
        d, _ = oracle.exact(g1, g2, c, directed=True)
        assert d == min(c[4], 2 * c[1] + 2 * c[4] + 2 * c[2] + c[5], c[1] + 2 * c[4] + c[2] + c[5])


def test_arc_labels_per_direction():
    """0 -> 1 labelled 1 and 1 -> 0 labelled 2, against the same arcs with the labels
    swapped: the identity relabels both arcs, the swap keeps both."""
    g1 = dg(2, [(0, 1), (1, 0)], el=[1, 2])
    g2 = dg(2, [(0, 1), (1, 0)], el=[2, 1])
    for c in ALL_COSTS:
        assert oracle.induced_cost(g1, g2, c, [0, 1], directed=True) == 2 * c[3]
        assert oracle.induced_cost(g1, g2, c, [1, 0], directed=True) == 0


def test_directed_path_and_cycle():
    """Path 0 -> 1 -> 2 against the 3-cycle 0 -> 1 -> 2 -> 0: the identity inserts the
    closing arc; the cheapest edit does the same (unit costs)."""
    g1, g2 = dg(3, [(0, 1), (1, 2)]), dg(3, [(0, 1), (1, 2), (2, 0)])
    assert oracle.induced_cost(g1, g2, UNIT, [0, 1, 2], directed=True) == 1
    assert oracle.induced_cost(g1, g2, UNIT, [2, 1, 0], directed=True) == 2 + 3
    assert oracle.exact(g1, g2, UNIT, directed=True)[0] == 1
    assert oracle.kbest(g1, g2, UNIT, 4, directed=True)[0] == 1


def test_rejects_self_loop_and_repeated_arc():
    with pytest.raises(oracle.OracleError):
        oracle.kbest(dg(2, [(0, 0)]), dg(2, []), UNIT, 2, directed=True)
    with pytest.raises(oracle.OracleError):
        oracle.kbest(dg(2, [(0, 1), (0, 1)]), dg(2, []), UNIT, 2, directed=True)
    # both directions of one pair are two distinct arcs: two deletions
    assert oracle.kbest(dg(2, [(0, 1), (1, 0)]), dg(2, []), UNIT, 2, directed=True)[0] == 2


# ------------------------------------------------ padded-permutation form
@pytest.mark.parametrize("seed", range(6))
def test_induced_cost_every_mapping(seed):
    g1 = tiny_directed(500 + seed, 0, 4, 0.45, 2, 2, n_min=1)
    g2 = tiny_directed(500 + seed, 1, 4, 0.45, 2, 2, n_min=1)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    n1, n2 = g1.n, g2.n
    for mp in itertools.product(range(-1, n2), repeat=n1):
        used = [x for x in mp if x >= 0]
        if len(used) != len(set(used)):
            continue
        want = _pins.qap_cost(g1, g2, c, _pins.perm_from_map(mp, n1, n2), directed=True)
        assert oracle.induced_cost(g1, g2, c, list(mp), directed=True) == want, mp


@pytest.mark.parametrize("seed", range(8))
def test_exact_against_permutations(seed):
    g1 = tiny_directed(520 + seed, 0, 4, 0.4, 2, 0 if seed % 2 else 2)
    g2 = tiny_directed(520 + seed, 1, 3, 0.5, 2, 0 if seed % 2 else 2)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    d, mp = oracle.exact(g1, g2, c, directed=True)
    assert d == _pins.qap_exact(g1, g2, c, directed=True)
    assert oracle.induced_cost(g1, g2, c, mp, directed=True) == d


# ------------------------------------------------ search from scratch
@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("K", [1, 2, 5, 17])
def test_kbest_against_scratch_beam(seed, K):
    g1 = tiny_directed(540 + seed, 0, 6, 0.35, 3, 0 if seed % 3 else 3)
    g2 = tiny_directed(540 + seed, 1, 6, 0.35, 3, 0 if seed % 3 else 3)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    for last in (False, True):
        d, mp = oracle.kbest(g1, g2, c, K, last_complete=last, directed=True)
        wd, wm = _pins.scratch_beam(g1, g2, c, K, last_complete=last, directed=True)
        assert (d, list(mp)) == (wd, wm), (seed, K, last)
        assert oracle.induced_cost(g1, g2, c, mp, directed=True) == d


# ------------------------------------------------ symmetric closure, reversal
@pytest.mark.parametrize("seed", range(8))
def test_symmetric_closure_is_undirected_with_doubled_edge_costs(seed):
    g1 = synth.random_small_graph(560 + seed, 0, 9, 0.4, 3, 0 if seed % 2 else 3, n_min=2)
    g2 = synth.random_small_graph(560 + seed, 1, 9, 0.4, 3, 0 if seed % 2 else 3, n_min=2)
    s1, s2 = symmetric_closure(g1), symmetric_closure(g2)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    c2 = doubled_edges(c)
    for K in (1, 3, 16, 64):
        for last in (False, True):
            d, mp = oracle.kbest(s1, s2, c, K, last_complete=last, directed=True)
            wd, wm = oracle.kbest(g1, g2, c2, K, last_complete=last)
            assert d == wd and np.array_equal(mp, wm), (K, last)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        mp = [-1] * g1.n
        tgt = rng.permutation(g2.n)
        for v in range(g1.n):
            if rng.random() < 0.7 and v < g2.n:
                mp[v] = int(tgt[v])
        assert oracle.induced_cost(s1, s2, c, mp, directed=True) == oracle.induced_cost(g1, g2, c2, mp)


@pytest.mark.parametrize("seed", range(8))
def test_reversing_every_arc_changes_nothing(seed):
    g1 = tiny_directed(580 + seed, 0, 12, 0.2, 3, 2, n_min=3)
    g2 = tiny_directed(580 + seed, 1, 12, 0.2, 3, 2, n_min=3)
    r1, r2 = reversed_graph(g1), reversed_graph(g2)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    for K in (1, 8, 64):
        for last in (False, True):
            a = oracle.kbest(g1, g2, c, K, last_complete=last, directed=True)
            b = oracle.kbest(r1, r2, c, K, last_complete=last, directed=True)
            assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_direction_matters():
    """A directed search is not the undirected one: on random directed pairs the two
    distances differ somewhere (guards against a mode flag that does nothing)."""
    differ = 0
    for k in range(20):
        g1 = tiny_directed(600, 2 * k, 8, 0.3, 2, n_min=4)
        g2 = tiny_directed(600, 2 * k + 1, 8, 0.3, 2, n_min=4)
        # the undirected reading needs simple graphs: drop the reverse arc of 2-cycles
        def und(g):
            seen, eu, ev = set(), [], []
            for a, b in zip(g.eu, g.ev):
                key = (min(a, b), max(a, b))
                if key not in seen:
                    seen.add(key)
                    eu.append(key[0])
                    ev.append(key[1])
            return Graph(g.n, g.vlabel, np.asarray(eu, np.int32), np.asarray(ev, np.int32), None)
        differ += oracle.kbest(g1, g2, UNIT, 8, directed=True)[0] != oracle.kbest(und(g1), und(g2), UNIT, 8)[0]
    assert differ >= 5


@pytest.mark.parametrize("seed", range(6))
def test_large_k_reaches_exact(seed):
    g1 = tiny_directed(620 + seed, 0, 5, 0.35, 2, 2, n_min=2)
    g2 = tiny_directed(620 + seed, 1, 5, 0.35, 2, 2, n_min=2)
    c = ALL_COSTS[seed % len(ALL_COSTS)]
    K = int(oracle.count_mappings(g1.n, g2.n)) + 1
    assert oracle.kbest(g1, g2, c, K, directed=True)[0] == oracle.exact(g1, g2, c, directed=True)[0]


def test_pairs_loop_matches_single_calls():
    w = synth.batch_directed_10_30(12)
    d, m, off = oracle.kbest_pairs(w.graphs, w.pairs, w.costs, 8, directed=True)
    for q, (a, b) in enumerate(w.pairs):
        g1, g2 = w.graphs.graph(int(a)), w.graphs.graph(int(b))
        dd, mm = oracle.kbest(g1, g2, w.costs, 8, directed=True)
        assert d[q] == dd and np.array_equal(m[off[q]:off[q] + g1.n], mm)
        assert oracle.induced_cost(g1, g2, w.costs, mm, directed=True) == dd
