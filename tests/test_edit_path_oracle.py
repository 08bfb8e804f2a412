"""Pins of the oracle's edit-path expansion (oracle.edit_path): for every mapping
of small pairs the operation costs sum to the mapping's edit cost (the padded
permutation brute force of tests/_pins.py), every vertex and edge of both graphs
appears in exactly one operation, and replaying the operations on g1 rebuilds g2
exactly (vertex and edge labels included).  The same holds for directed graphs,
with arcs in place of edges."""
import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from tests import _pins

COSTS = [synth.UNIT_COSTS, synth.PAPER_COSTS, (3, 2, 5, 9, 1, 2), (4, 12, 12, 1, 10, 10)]


def labelled_edges(g, directed=False):
    el = g.elabel if getattr(g, "elabel", None) is not None else [0] * len(g.eu)
    if directed:
        return {(int(a), int(b)): int(l) for a, b, l in zip(g.eu, g.ev, el)}
    return {(min(int(a), int(b)), max(int(a), int(b))): int(l) for a, b, l in zip(g.eu, g.ev, el)}


def replay(g1, g2, ops, costs, directed=False):
    """Apply the operations to g1; return the resulting labelled graph in g2's
    vertex names, and check that each element is touched exactly once and
    that each operation carries its own cost."""
    E1 = labelled_edges(g1, directed)
    E2 = labelled_edges(g2, directed)
    seen_v1, seen_v2, seen_e1, seen_e2 = set(), set(), set(), set()
    names = {}
    vlab = {}
    edges = dict(E1)
    for kind, a, b, c, d, cost in ops:
        if kind == 0:                       # vertex substitution: g1 vertex a becomes g2 vertex b
            assert a not in seen_v1 and b not in seen_v2
            seen_v1.add(a), seen_v2.add(b)
            names[a] = b
            vlab[b] = int(g2.vlabel[b])
            assert cost == (0 if int(g1.vlabel[a]) == int(g2.vlabel[b]) else costs[0])
        elif kind == 1:                     # vertex deletion
            assert a not in seen_v1 and cost == costs[1]
            seen_v1.add(a)
        elif kind == 2:                     # vertex insertion
            assert b not in seen_v2 and cost == costs[2]
            seen_v2.add(b)
            vlab[b] = int(g2.vlabel[b])
        elif kind == 3:                     # edge substitution: g1 edge (a, b) becomes g2 edge (c, d)
            assert (a, b) not in seen_e1 and (c, d) not in seen_e2
            seen_e1.add((a, b)), seen_e2.add((c, d))
            assert cost == (0 if E1[(a, b)] == E2[(c, d)] else costs[3])
            edges[(a, b)] = E2[(c, d)]
        elif kind == 4:                     # edge deletion
            assert (a, b) not in seen_e1 and cost == costs[4]
            seen_e1.add((a, b))
            del edges[(a, b)]
        elif kind == 5:                     # edge insertion
            assert (c, d) not in seen_e2 and cost == costs[5]
            seen_e2.add((c, d))
    assert seen_v1 == set(range(int(g1.n))) and seen_v2 == set(range(int(g2.n)))
    assert seen_e1 == set(E1) and seen_e2 == set(E2)
    out = {}
    for (a, b), l in edges.items():
        x, y = names[a], names[b]                # surviving g1 edges have both ends substituted
        out[(x, y) if directed else (min(x, y), max(x, y))] = l
    for kind, a, b, c, d, cost in ops:
        if kind == 5:
            out[(c, d)] = E2[(c, d)]
    return vlab, out


@pytest.mark.parametrize("costs", COSTS)
def test_every_mapping_of_small_pairs(costs):
    """Degenerate pairs (an empty or edgeless graph) and pairs with edges on both sides, so
    that edges substituted under order-reversing mappings and edge insertions occur."""
    gs = [synth.random_small_graph(101, k, 4, 0.6, 2, 3) for k in range(8)]
    gs += [synth.random_small_graph(102, k, 4, 0.7, 2, 3, n_min=3) for k in range(6)]
    reversing = inserted = 0
    for g1, g2 in zip(gs[0::2], gs[1::2]):
        E2 = labelled_edges(g2)
        for mp in _pins.all_mappings(int(g1.n), int(g2.n)):
            ops = oracle.edit_path(g1, g2, costs, mp)
            total = sum(op[5] for op in ops)
            assert total == _pins.qap_cost(g1, g2, costs, _pins.perm_from_map(mp, int(g1.n), int(g2.n)))
            vlab, edges = replay(g1, g2, ops, costs)
            assert vlab == {u: int(g2.vlabel[u]) for u in range(int(g2.n))}
            assert edges == E2
            reversing += sum(1 for op in ops if op[0] == 3 and mp[op[1]] > mp[op[2]])
            inserted += sum(1 for op in ops if op[0] == 5)
    assert reversing > 0 and inserted > 0


@pytest.mark.parametrize("costs", COSTS)
def test_every_mapping_of_small_directed_pairs(costs):
    """Both graphs of each pair carry arcs, so substitutions onto arcs whose image runs from
    a higher to a lower g2 index, and insertions of uncovered arcs, both occur."""
    gs = [synth.directed_graph(105, k, 2, 4, 0.5, 0.5, 2, 3) for k in range(8)]
    reversed_images = inserted = 0
    for g1, g2 in zip(gs[0::2], gs[1::2]):
        E2 = labelled_edges(g2, True)
        for mp in _pins.all_mappings(int(g1.n), int(g2.n)):
            ops = oracle.edit_path(g1, g2, costs, mp, directed=True)
            total = sum(op[5] for op in ops)
            assert total == _pins.qap_cost(g1, g2, costs, _pins.perm_from_map(mp, int(g1.n), int(g2.n)),
                                           directed=True)
            vlab, edges = replay(g1, g2, ops, costs, directed=True)
            assert vlab == {u: int(g2.vlabel[u]) for u in range(int(g2.n))}
            assert edges == E2
            reversed_images += sum(1 for op in ops if op[0] == 3 and op[3] > op[4])
            inserted += sum(1 for op in ops if op[0] == 5)
    assert reversed_images > 0 and inserted > 0


def test_order_and_cost_of_each_operation():
    gs = [synth.random_small_graph(103, k, 12, 0.4, 3, 4) for k in range(10)]
    rng = np.random.default_rng(5)
    c = (3, 2, 5, 9, 1, 2)
    for g1, g2 in zip(gs[0::2], gs[1::2]):
        n1, n2 = int(g1.n), int(g2.n)
        perm = rng.permutation(n2)
        mp = [int(perm[v]) if v < n2 and rng.random() < 0.7 else -1 for v in range(n1)]
        ops = oracle.edit_path(g1, g2, c, mp)
        kinds = [op[0] for op in ops]
        assert kinds == sorted(kinds, key=lambda k: {0: 0, 1: 0, 2: 1, 3: 2, 4: 2, 5: 3}[k])
        assert [op[1] for op in ops[:n1]] == list(range(n1))
        ins = [op[2] for op in ops if op[0] == 2]
        assert ins == sorted(ins) and len(ins) == n2 - sum(1 for x in mp if x >= 0)
        e1 = [(op[1], op[2]) for op in ops if op[0] in (3, 4)]
        assert e1 == sorted(labelled_edges(g1))
        e2 = [(op[3], op[4]) for op in ops if op[0] == 5]
        assert e2 == sorted(e2)
        assert sum(op[5] for op in ops) == oracle.induced_cost(g1, g2, c, mp)
