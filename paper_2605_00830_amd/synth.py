"""Seeded synthetic graph workloads.

This module only draws graphs and pairs; it holds none of the edit-distance
arithmetic.  Every random number comes from one counter-based generator
(the SplitMix64 finaliser of Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) keyed by
(seed, graph index, stream tag) and indexed by a counter, so a graph's
content depends only on its own key: generation is order-independent and
identical on every machine (integer arithmetic only; floats are formed from
the top 53 bits).

Workloads follow the shapes of the paper's evaluation (Sec. 5): random
Erdos-Renyi graphs with uniform node labels and molecule-shaped sparse
labelled graphs standing in for the chemistry datasets, which are not used
here.  Graphs are undirected and simple (Sec. 2.1).
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _mix_int(z: int) -> int:
    z &= _MASK
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def _mix_arr(z: np.ndarray) -> np.ndarray:
    # uint64 array arithmetic wraps modulo 2**64, as the finaliser requires.
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, index: int, tag: int) -> int:
    """64-bit key of the stream (seed, index, tag)."""
    k = _mix_int(seed * _GAMMA + 0x1234567)
    k = _mix_int(k + (index + 1) * _GAMMA)
    return _mix_int(k + (tag + 1) * _GAMMA)


def uniforms(seed: int, index: int, tag: int, count: int) -> np.ndarray:
    """`count` doubles in [0, 1): element c is mix(key + (c+1)*gamma) >> 11 / 2**53."""
    if count <= 0:
        return np.zeros(0, dtype=np.float64)
    key = np.uint64(stream_key(seed, index, tag))
    ctr = np.arange(1, count + 1, dtype=np.uint64) * np.uint64(_GAMMA)
    bits = _mix_arr(ctr + key) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def _uint_below(u: np.ndarray, bound: int) -> np.ndarray:
    return np.minimum((u * bound).astype(np.int64), bound - 1)


# --------------------------------------------------------------------------
# Graph containers
# --------------------------------------------------------------------------

@dataclass
class Graph:
    """One undirected simple labelled graph (Sec. 2.1): vertices 0..n-1.
    A directed graph uses the same fields, edge k being the arc eu[k] -> ev[k]."""
    n: int
    vlabel: np.ndarray                      # int32 [n]
    eu: np.ndarray                          # int32 [m], eu < ev (undirected)
    ev: np.ndarray                          # int32 [m]
    elabel: Optional[np.ndarray] = None     # int32 [m] or None (all edges label 0)

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])


@dataclass
class GraphSet:
    """Many graphs stored as concatenated arrays (vertex and edge offsets)."""
    n: np.ndarray          # int32 [G]
    m: np.ndarray          # int32 [G]
    voff: np.ndarray       # int64 [G+1]
    eoff: np.ndarray       # int64 [G+1]
    vlabel: np.ndarray     # int32 [sum n]
    eu: np.ndarray         # int32 [sum m]
    ev: np.ndarray         # int32 [sum m]
    elabel: Optional[np.ndarray]  # int32 [sum m] or None

    def __len__(self) -> int:
        return int(self.n.shape[0])

    def slice(self, lo: int, hi: int) -> "GraphSet":
        """Graphs lo..hi-1 as a GraphSet of their own (arrays are copied)."""
        a, b = int(self.voff[lo]), int(self.voff[hi])
        c, d = int(self.eoff[lo]), int(self.eoff[hi])
        el = None if self.elabel is None else self.elabel[c:d].copy()
        return GraphSet(self.n[lo:hi].copy(), self.m[lo:hi].copy(), self.voff[lo:hi + 1] - a,
                        self.eoff[lo:hi + 1] - c, self.vlabel[a:b].copy(), self.eu[c:d].copy(),
                        self.ev[c:d].copy(), el)

    def graph(self, i: int) -> Graph:
        a, b = int(self.voff[i]), int(self.voff[i + 1])
        c, d = int(self.eoff[i]), int(self.eoff[i + 1])
        el = None if self.elabel is None else self.elabel[c:d]
        return Graph(int(self.n[i]), self.vlabel[a:b], self.eu[c:d], self.ev[c:d], el)

    @staticmethod
    def from_graphs(graphs: Sequence[Graph]) -> "GraphSet":
        G = len(graphs)
        n = np.array([g.n for g in graphs], dtype=np.int32)
        m = np.array([g.m for g in graphs], dtype=np.int32)
        voff = np.zeros(G + 1, dtype=np.int64)
        eoff = np.zeros(G + 1, dtype=np.int64)
        np.cumsum(n, out=voff[1:])
        np.cumsum(m, out=eoff[1:])

        def cat(parts, dt=np.int32):
            parts = [np.asarray(p, dtype=dt) for p in parts]
            return np.concatenate(parts) if parts else np.zeros(0, dtype=dt)

        vl = cat([g.vlabel for g in graphs])
        eu = cat([g.eu for g in graphs])
        ev = cat([g.ev for g in graphs])
        if any(g.elabel is not None for g in graphs):
            el = cat([g.elabel if g.elabel is not None else np.zeros(g.m, np.int32)
                      for g in graphs])
        else:
            el = None
        return GraphSet(n, m, voff, eoff, vl, eu, ev, el)


# --------------------------------------------------------------------------
# Generators
# --------------------------------------------------------------------------

def er_graph(seed: int, index: int, n_lo: int, n_hi: int, p_lo: float, p_hi: float,
             n_vlabels: int) -> Graph:
    """Erdos-Renyi G(n, p): n ~ U{n_lo..n_hi}, p ~ U[p_lo, p_hi], labels ~ U{0..L-1}.

    Stream tags: 0 = (n, p), 1 = vertex labels, 2 = one draw per unordered
    vertex pair in row-major (a < b) order; the pair is an edge iff draw < p.
    """
    u = uniforms(seed, index, 0, 2)
    n = n_lo + int(_uint_below(u[:1], n_hi - n_lo + 1)[0])
    p = p_lo + float(u[1]) * (p_hi - p_lo)
    vl = _uint_below(uniforms(seed, index, 1, n), n_vlabels).astype(np.int32)
    a, b = np.triu_indices(n, 1)
    keep = uniforms(seed, index, 2, a.shape[0]) < p
    return Graph(n, vl, a[keep].astype(np.int32), b[keep].astype(np.int32), None)


def directed_graph(seed: int, index: int, n_lo: int, n_hi: int, p_lo: float, p_hi: float,
                   n_vlabels: int, n_elabels: int = 0) -> Graph:
    """Directed G(n, p): n ~ U{n_lo..n_hi}, p ~ U[p_lo, p_hi], vertex labels ~ U{0..L-1}.

    Stream tags: 0 = (n, p), 1 = vertex labels, 2 = one draw per ordered pair
    (a, b), a != b, in row-major order; the arc a -> b exists iff draw < p (so
    both arcs of a pair can exist); 5 = arc labels ~ U{0..n_elabels-1}.
    """
    u = uniforms(seed, index, 0, 2)
    n = n_lo + int(_uint_below(u[:1], n_hi - n_lo + 1)[0])
    p = p_lo + float(u[1]) * (p_hi - p_lo)
    vl = _uint_below(uniforms(seed, index, 1, n), n_vlabels).astype(np.int32)
    a, b = np.nonzero(~np.eye(n, dtype=bool))
    keep = uniforms(seed, index, 2, a.shape[0]) < p
    g = Graph(n, vl, a[keep].astype(np.int32), b[keep].astype(np.int32), None)
    if n_elabels > 0:
        g.elabel = _uint_below(uniforms(seed, index, 5, g.m), n_elabels).astype(np.int32)
    return g


def _prufer_tree(seq: np.ndarray, n: int) -> List[Tuple[int, int]]:
    """Decode a Pruefer sequence (length n-2) into the n-1 edges of its labelled tree."""
    degree = [1] * n
    for x in seq:
        degree[int(x)] += 1
    leaves = [v for v in range(n) if degree[v] == 1]
    heapq.heapify(leaves)
    edges = []
    for x in seq:
        x = int(x)
        leaf = heapq.heappop(leaves)
        edges.append((min(leaf, x), max(leaf, x)))
        degree[x] -= 1
        if degree[x] == 1:
            heapq.heappush(leaves, x)
    a = heapq.heappop(leaves)
    b = heapq.heappop(leaves)
    edges.append((min(a, b), max(a, b)))
    return edges


MOLECULE_VLABEL_P = np.array([0.6, 0.15, 0.1] + [0.15 / 7] * 7, dtype=np.float64)


def molecule_graph(seed: int, index: int, n_lo: int = 10, n_hi: int = 70,
                   extra_frac: float = 0.1, n_elabels: int = 3) -> Graph:
    """Sparse connected molecule-shaped graph.

    A uniform random labelled tree (decoded from a uniform Pruefer sequence)
    plus round(extra_frac * (n - 1)) extra edges chosen uniformly among the
    non-edges (mean degree about 2.2).  Vertex labels follow the skewed
    distribution MOLECULE_VLABEL_P over 10 labels; edge labels are uniform
    over {0 .. n_elabels-1}.

    Stream tags: 0 = n, 1 = Pruefer sequence, 3 = extra-edge draws,
    4 = vertex labels, 5 = edge labels.
    """
    n = n_lo + int(_uint_below(uniforms(seed, index, 0, 1), n_hi - n_lo + 1)[0])
    seq = _uint_below(uniforms(seed, index, 1, n - 2), n)
    tree = _prufer_tree(seq, n)
    adj = np.zeros((n, n), dtype=bool)
    for x, y in tree:
        adj[x, y] = True
    k = int(np.floor(extra_frac * (n - 1) + 0.5))
    if k > 0:
        a, b = np.triu_indices(n, 1)
        free = ~adj[a, b]
        ca, cb = a[free], b[free]          # the non-edges in row-major order
        draws = uniforms(seed, index, 3, k)
        # partial Fisher-Yates over the non-edge list
        for t in range(k):
            j = t + int(_uint_below(draws[t:t + 1], len(ca) - t)[0])
            ca[t], ca[j] = ca[j], ca[t]
            cb[t], cb[j] = cb[j], cb[t]
            adj[ca[t], cb[t]] = True
    eu, ev = np.nonzero(np.triu(adj, 1))
    eu = eu.astype(np.int32)
    ev = ev.astype(np.int32)
    cum = np.cumsum(MOLECULE_VLABEL_P)
    cum[-1] = 1.0
    vl = np.searchsorted(cum, uniforms(seed, index, 4, n), side="right").astype(np.int32)
    vl = np.minimum(vl, len(MOLECULE_VLABEL_P) - 1).astype(np.int32)
    elab = _uint_below(uniforms(seed, index, 5, eu.shape[0]), n_elabels).astype(np.int32)
    return Graph(n, vl, eu, ev, elab)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

UNIT_COSTS = (1, 1, 1, 1, 1, 1)          # vsub, vdel, vins, esub, edel, eins
PAPER_COSTS = (2, 4, 4, 1, 2, 2)         # the paper's default setting (Sec. 5)


@dataclass
class Workload:
    name: str
    graphs: GraphSet
    pairs: np.ndarray                  # int64 [P, 2]: (source g1, target g2) ids
    costs: Tuple[int, int, int, int, int, int]
    K: int
    meta: dict = field(default_factory=dict)


def _er_pairs(seed, npairs, n_lo, n_hi, p_lo, p_hi, nl) -> GraphSet:
    return GraphSet.from_graphs([er_graph(seed, i, n_lo, n_hi, p_lo, p_hi, nl)
                                 for i in range(2 * npairs)])


def pair_er_8x9() -> Workload:
    """One ER pair, n1=8, n2=9, p=0.3, 4 vertex labels, unit costs, K=16 (seed 1)."""
    g1 = er_graph(1, 0, 8, 8, 0.3, 0.3, 4)
    g2 = er_graph(1, 1, 9, 9, 0.3, 0.3, 4)
    return Workload("pair_er_8x9_k16", GraphSet.from_graphs([g1, g2]),
                    np.array([[0, 1]], dtype=np.int64), UNIT_COSTS, 16)


def batch_er_10_30(npairs: int = 4096) -> Workload:
    """npairs ER pairs, n ~ U{10..30}, p ~ U[0.1,0.3], 5 labels, unit costs, K=64 (seed 2)."""
    gs = _er_pairs(2, npairs, 10, 30, 0.1, 0.3, 5)
    pairs = np.stack([np.arange(0, 2 * npairs, 2), np.arange(1, 2 * npairs, 2)], 1)
    return Workload(f"batch_er_n10-30_p0.1-0.3_{npairs}pairs_k64", gs,
                    pairs.astype(np.int64), UNIT_COSTS, 64)


def query_molecule_10_70(ndb: int = 10000) -> Workload:
    """One molecule-shaped query (g1) against ndb molecule-shaped graphs, paper costs, K=128 (seed 3).

    Graph 0 is the query; graphs 1..ndb form the database.
    """
    gs = GraphSet.from_graphs([molecule_graph(3, i) for i in range(ndb + 1)])
    pairs = np.stack([np.zeros(ndb, np.int64), np.arange(1, ndb + 1, dtype=np.int64)], 1)
    return Workload(f"query_molecule_n10-70_1x{ndb}_k128", gs, pairs, PAPER_COSTS, 128)


def batch_molecule_k64(npairs: int = 10000) -> Workload:
    """npairs disjoint pairs of molecule-shaped graphs (n 10..70; the molecule graphs of
    query_molecule_10_70, seed 3), unit costs, K=64: the molecule half of the serving mix."""
    gs = GraphSet.from_graphs([molecule_graph(3, i) for i in range(1, 2 * npairs + 1)])
    pairs = np.stack([np.arange(0, 2 * npairs, 2), np.arange(1, 2 * npairs, 2)], 1)
    return Workload(f"batch_molecule_n10-70_{npairs}pairs_k64", gs, pairs.astype(np.int64), UNIT_COSTS, 64)


def batch_directed_10_30(npairs: int = 4096) -> Workload:
    """npairs directed G(n, p) pairs, n ~ U{10..30}, p ~ U[0.05,0.15] per ordered pair (about the
    arc count of batch_er_10_30's edges), 5 vertex labels, unit costs, K=64 (seed 8)."""
    gs = GraphSet.from_graphs([directed_graph(8, i, 10, 30, 0.05, 0.15, 5) for i in range(2 * npairs)])
    pairs = np.stack([np.arange(0, 2 * npairs, 2), np.arange(1, 2 * npairs, 2)], 1)
    return Workload(f"batch_directed_n10-30_p0.05-0.15_{npairs}pairs_k64", gs,
                    pairs.astype(np.int64), UNIT_COSTS, 64)


def stress_er_100_500(npairs: int = 256) -> Workload:
    """npairs ER pairs, n ~ U{100..500}, p ~ U[0.05,0.5], 8 labels, unit costs, K=256 (seed 4)."""
    gs = _er_pairs(4, npairs, 100, 500, 0.05, 0.5, 8)
    pairs = np.stack([np.arange(0, 2 * npairs, 2), np.arange(1, 2 * npairs, 2)], 1)
    return Workload(f"stress_er_n100-500_p0.05-0.5_{npairs}pairs_k256", gs,
                    pairs.astype(np.int64), UNIT_COSTS, 256)


def pair_er_large_k(n: int, seed: int) -> Workload:
    """One ER pair for the single-pair large-K search: n vertices each, p = 0.4, 4 vertex
    labels, no edge labels, the paper's cost setting 1 (seed 6 for n = 20, 7 for n = 500).

    The shapes of the paper's runtime-versus-K experiment (two 20-vertex graphs) and of its
    runtime-versus-size experiment (density 0.4, K = 5000); the paper states neither labels
    nor seeds, so the labels are a reading.
    """
    g1 = er_graph(seed, 0, n, n, 0.4, 0.4, 4)
    g2 = er_graph(seed, 1, n, n, 0.4, 0.4, 4)
    return Workload(f"pair_er_n{n}_p0.4", GraphSet.from_graphs([g1, g2]),
                    np.array([[0, 1]], dtype=np.int64), PAPER_COSTS, 0)


def mix_graph(seed: int, index: int) -> Graph:
    """Serving-mix graph: 49.5% small ER (n 10..30), 49.5% molecule (n 10..70), 1% large ER (n 100..500)."""
    u = float(uniforms(seed, index, 9, 1)[0])
    if u < 0.495:
        return er_graph(seed, index, 10, 30, 0.1, 0.3, 5)
    if u < 0.99:
        return molecule_graph(seed, index)
    return er_graph(seed, index, 100, 500, 0.05, 0.5, 8)


def serve_mix(ndb: int = 100000, nqueries: int = 100000) -> Workload:
    """Serving stream: a database of ndb mix graphs and nqueries (query graph, target id) pairs, K=64, unit costs (seed 5).

    Graphs 0..ndb-1 are the database; graph ndb+q is query q's graph.
    """
    graphs = [mix_graph(5, i) for i in range(ndb)]
    graphs += [mix_graph(5, 10_000_000 + q) for q in range(nqueries)]
    tgt = _uint_below(uniforms(5, 0, 10, nqueries), ndb)
    pairs = np.stack([np.arange(ndb, ndb + nqueries, dtype=np.int64), tgt], 1)
    return Workload(f"serve_mix_db{ndb}_q{nqueries}_k64", GraphSet.from_graphs(graphs),
                    pairs.astype(np.int64), UNIT_COSTS, 64, {"ndb": ndb})


def directed_mix_graph(seed: int, index: int) -> Graph:
    """Directed serving-mix graph: 49.5% small (n 10..30, arc p 0.05..0.15), 49.5% mid
    (n 33..70, p 0.02..0.06, 3 arc labels), 1% large (n 100..256, p 0.01..0.05, 3 arc labels)."""
    u = float(uniforms(seed, index, 9, 1)[0])
    if u < 0.495:
        return directed_graph(seed, index, 10, 30, 0.05, 0.15, 5, 3)
    if u < 0.99:
        return directed_graph(seed, index, 33, 70, 0.02, 0.06, 5, 3)
    return directed_graph(seed, index, 100, 256, 0.01, 0.05, 5, 3)


def serve_mix_directed(ndb: int = 100000, nqueries: int = 100000) -> Workload:
    """Directed serving stream, laid out as serve_mix: ndb directed mix graphs, then one
    query graph per query, targets uniform over the database; K=64, unit costs (seed 9)."""
    graphs = [directed_mix_graph(9, i) for i in range(ndb)]
    graphs += [directed_mix_graph(9, 10_000_000 + q) for q in range(nqueries)]
    tgt = _uint_below(uniforms(9, 0, 10, nqueries), ndb)
    pairs = np.stack([np.arange(ndb, ndb + nqueries, dtype=np.int64), tgt], 1)
    return Workload(f"serve_mix_directed_db{ndb}_q{nqueries}_k64", GraphSet.from_graphs(graphs),
                    pairs.astype(np.int64), UNIT_COSTS, 64, {"ndb": ndb, "directed": True})


def random_small_graph(seed: int, index: int, n_max: int, p: float, n_vlabels: int,
                       n_elabels: int = 0, n_min: int = 0) -> Graph:
    """Tiny ER graph for property tests: n ~ U{n_min..n_max}; optional uniform edge labels."""
    g = er_graph(seed, index, n_min, n_max, p, p, n_vlabels)
    if n_elabels > 0:
        g.elabel = _uint_below(uniforms(seed, index, 5, g.m), n_elabels).astype(np.int32)
    return g
