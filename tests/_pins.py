"""Independent pure-Python computations that pin the oracle.

None of this shares code with oracle/ged_oracle.c; each function reaches the
same quantity by a different route:

* qap_cost / qap_exact: the quadratic-assignment form of GED -- both graphs
  padded with epsilon vertices to n1+n2, a permutation of the padded vertex
  set, vertex and edge costs read off position by position (Sec. 2.2-2.4 of
  the paper written as one formula over the padded adjacency).
* scratch_beam: the K-Best search of Alg. 1 where every child's partial edit
  distance is recomputed from scratch as the cost of all edit operations in
  its path (Sec. 4.2.2), instead of the incremental implied-edge
  scan, and ranking uses the child's mapping tuple itself (deleted = n2) for
  the generation-order tie-break; optionally with the complete-then-minimum
  last level, scored by the padded-permutation cost of each complete path.

Each takes `directed`: edge k is then the arc eu[k] -> ev[k], and every loop
over unordered vertex pairs runs over ordered pairs instead (one edit
operation per arc).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

VSUB, VDEL, VINS, ESUB, EDEL, EINS = range(6)


def edge_dict(g, directed: bool = False) -> Dict[Tuple[int, int], int]:
    el = g.elabel if getattr(g, "elabel", None) is not None else [0] * len(g.eu)
    d = {}
    for a, b, l in zip(g.eu, g.ev, el):
        a, b, l = int(a), int(b), int(l)
        d[(a, b)] = l
        if not directed:
            d[(b, a)] = l
    return d


def _pairs(idx: Sequence[int], directed: bool):
    """Unordered pairs (i < j) of idx, or every ordered pair i != j."""
    if directed:
        return [(i, j) for i in idx for j in idx if i != j]
    return [(idx[a], idx[b]) for a in range(len(idx)) for b in range(a + 1, len(idx))]


def qap_cost(g1, g2, c: Sequence[int], perm: Sequence[int], directed: bool = False) -> int:
    """Cost of a permutation of the padded vertex set (size n1+n2).

    Position i < n1 is g1 vertex i, position i >= n1 an epsilon; target
    index t < n2 is g2 vertex t, t >= n2 an epsilon.
    """
    n1, n2 = int(g1.n), int(g2.n)
    N = n1 + n2
    E1, E2 = edge_dict(g1, directed), edge_dict(g2, directed)
    cost = 0
    for i in range(N):
        t = perm[i]
        if i < n1 and t < n2:
            cost += c[VSUB] if int(g1.vlabel[i]) != int(g2.vlabel[t]) else 0
        elif i < n1:
            cost += c[VDEL]
        elif t < n2:
            cost += c[VINS]
    for i, j in _pairs(list(range(N)), directed):
        e1 = E1.get((i, j)) if (i < n1 and j < n1) else None
        a, b = perm[i], perm[j]
        e2 = E2.get((a, b)) if (a < n2 and b < n2) else None
        if e1 is not None and e2 is not None:
            cost += c[ESUB] if e1 != e2 else 0
        elif e1 is not None:
            cost += c[EDEL]
        elif e2 is not None:
            cost += c[EINS]
    return cost


def perm_from_map(mapping: Sequence[int], n1: int, n2: int) -> List[int]:
    """Extend a mapping (-1 = deleted) to a padded permutation."""
    perm = [0] * (n1 + n2)
    used = set(int(x) for x in mapping if int(x) >= 0)
    free_eps_targets = iter(range(n2, n2 + n1))
    for i in range(n1):
        perm[i] = int(mapping[i]) if int(mapping[i]) >= 0 else next(free_eps_targets)
    rest_targets = [t for t in range(n2) if t not in used] + list(free_eps_targets)
    for k, i in enumerate(range(n1, n1 + n2)):
        perm[i] = rest_targets[k]
    return perm


def qap_exact(g1, g2, c: Sequence[int], directed: bool = False) -> int:
    n1, n2 = int(g1.n), int(g2.n)
    return min(qap_cost(g1, g2, c, p, directed) for p in itertools.permutations(range(n1 + n2)))


def partial_cost(g1, g2, c, phi: Sequence[int], directed: bool = False) -> int:
    """Cost of all edit operations on the path phi (g1 vertices 0..len(phi)-1 edited)."""
    E1, E2 = edge_dict(g1, directed), edge_dict(g2, directed)
    k = len(phi)
    cost = 0
    img = {}
    for v in range(k):
        t = phi[v]
        if t < 0:
            cost += c[VDEL]
        else:
            img[t] = v
            cost += c[VSUB] if int(g1.vlabel[v]) != int(g2.vlabel[t]) else 0
    for a, b in _pairs(list(range(k)), directed):
        e1 = E1.get((a, b))
        if e1 is None:
            continue
        x, y = phi[a], phi[b]
        e2 = E2.get((x, y)) if (x >= 0 and y >= 0) else None
        if e2 is None:
            cost += c[EDEL]
        elif e2 != e1:
            cost += c[ESUB]
    for x, y in _pairs(sorted(img), directed):
        if (x, y) in E2 and (img[x], img[y]) not in E1:
            cost += c[EINS]
    return cost


def scratch_beam(g1, g2, c, K: int, last_complete: bool = False,
                 directed: bool = False, count: Optional[List[int]] = None) -> Tuple[int, List[int]]:
    """last_complete: at the last level every child is scored by the cost of its
    complete edit path (the padded-permutation form, qap_cost) and the least
    (cost, mapping tuple) is returned.  count (a list, may be None) gets one
    entry per level: the number of children generated there."""
    n1, n2 = int(g1.n), int(g2.n)
    E2 = edge_dict(g2, directed)

    def key(phi):  # lexicographic key with deletion after every g2 vertex
        return tuple(n2 if t < 0 else t for t in phi)

    beam: List[Tuple[int, ...]] = [()]
    for i in range(n1):
        children = []
        for phi in beam:
            used = {t for t in phi if t >= 0}
            for u in list(range(n2)) + [-1]:
                if u >= 0 and u in used:
                    continue
                ch = phi + (u,)
                children.append((partial_cost(g1, g2, c, ch, directed), key(ch), ch))
        if count is not None:
            count.append(len(children))
        if last_complete and i == n1 - 1:
            best_c = min((qap_cost(g1, g2, c, perm_from_map(ch, n1, n2), directed), key(ch), ch)
                         for _, _, ch in children)
            return best_c[0], list(best_c[2])
        children.sort(key=lambda x: (x[0], x[1]))
        kept = children[:K]
        kept.sort(key=lambda x: x[1])
        beam = [x[2] for x in kept]
    best: Optional[Tuple[int, Tuple[int, ...], Tuple[int, ...]]] = None
    for phi in beam:
        used = {t for t in phi if t >= 0}
        total = partial_cost(g1, g2, c, phi, directed) + c[VINS] * (n2 - len(used))
        for x, y in _pairs(list(range(n2)), directed):
            if (x, y) in E2 and (x not in used or y not in used):
                total += c[EINS]
        cand = (total, key(phi), phi)
        if best is None or cand[:2] < best[:2]:
            best = cand
    return best[0], list(best[2])


def to_networkx(g):
    import networkx as nx
    G = nx.Graph()
    for v in range(int(g.n)):
        G.add_node(v, label=int(g.vlabel[v]))
    el = g.elabel if getattr(g, "elabel", None) is not None else [0] * len(g.eu)
    for a, b, l in zip(g.eu, g.ev, el):
        G.add_edge(int(a), int(b), label=int(l))
    return G


def networkx_ged(g1, g2, c) -> int:
    import networkx as nx
    return int(round(nx.graph_edit_distance(
        to_networkx(g1), to_networkx(g2),
        node_subst_cost=lambda a, b: 0 if a["label"] == b["label"] else c[VSUB],
        node_del_cost=lambda a: c[VDEL],
        node_ins_cost=lambda a: c[VINS],
        edge_subst_cost=lambda a, b: 0 if a["label"] == b["label"] else c[ESUB],
        edge_del_cost=lambda a: c[EDEL],
        edge_ins_cost=lambda a: c[EINS])))


# ---------------------------------------------------------------------------
# Bipartite K-best assignments: every vertex mapping with its bipartite
# (Riesen-Bunke) assignment cost, the local edge term found by brute force
# over the incident edges instead of a closed form.

def incident_labels(g) -> List[List[int]]:
    el = g.elabel if getattr(g, "elabel", None) is not None else [0] * len(g.eu)
    out: List[List[int]] = [[] for _ in range(int(g.n))]
    for a, b, l in zip(g.eu, g.ev, el):
        out[int(a)].append(int(l))
        out[int(b)].append(int(l))
    return out


def edge_assignment_cost(A: Sequence[int], B: Sequence[int], c: Sequence[int]) -> int:
    """Least cost of editing the edge-label list A into B: every injective
    partial matching of A into B tried (matched pairs cost esub when the labels
    differ, unmatched A edges edel, unmatched B edges eins)."""
    best = None
    nA, nB = len(A), len(B)
    for k in range(min(nA, nB) + 1):
        for sa in itertools.combinations(range(nA), k):
            for sb in itertools.permutations(range(nB), k):
                cost = sum(c[ESUB] if A[x] != B[y] else 0 for x, y in zip(sa, sb))
                cost += c[EDEL] * (nA - k) + c[EINS] * (nB - k)
                if best is None or cost < best:
                    best = cost
    return 0 if best is None else best


def all_mappings(n1: int, n2: int):
    """Every vertex mapping g1 -> g2 (-1 = deleted), injective on g2."""
    def rec(i, used, cur):
        if i == n1:
            yield list(cur)
            return
        for t in range(n2):
            if t not in used:
                used.add(t)
                cur.append(t)
                yield from rec(i + 1, used, cur)
                cur.pop()
                used.discard(t)
        cur.append(-1)
        yield from rec(i + 1, used, cur)
        cur.pop()
    yield from rec(0, set(), [])


def bipartite_cost(g1, g2, c: Sequence[int], mapping: Sequence[int], inc1=None, inc2=None) -> int:
    """Assignment cost of a mapping in the square bipartite matrix: substituted
    pairs (label cost + least incident-edge assignment), deleted g1 vertices
    with their edges, inserted g2 vertices with their edges."""
    inc1 = incident_labels(g1) if inc1 is None else inc1
    inc2 = incident_labels(g2) if inc2 is None else inc2
    used = set()
    cost = 0
    for i, t in enumerate(mapping):
        t = int(t)
        if t >= 0:
            used.add(t)
            cost += c[VSUB] if int(g1.vlabel[i]) != int(g2.vlabel[t]) else 0
            cost += edge_assignment_cost(inc1[i], inc2[t], c)
        else:
            cost += c[VDEL] + c[EDEL] * len(inc1[i])
    for t in range(int(g2.n)):
        if t not in used:
            cost += c[VINS] + c[EINS] * len(inc2[t])
    return cost
