"""CPU oracle for the K-Best graph edit distance search -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it; see ged_oracle.c (the paper's
K-Best tree search) and bipartite_oracle.c (the bipartite K-best-assignment
variant) for the definitions they follow and what they cite.

Functions take `Graph` objects from paper_2605_00830_amd.synth (or anything
with n, vlabel, eu, ev, elabel) and a 6-tuple of costs
(vsub, vdel, vins, esub, edel, eins).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "ged_oracle.c"), os.path.join(_HERE, "bipartite_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ETOOBIG = 0, 1, 2, 3


class OracleError(RuntimeError):
    pass


def _stale() -> bool:
    return not os.path.exists(_LIB_PATH) or any(os.path.getmtime(_LIB_PATH) < os.path.getmtime(f) for f in _SRCS)


def build(force: bool = True) -> str:
    """Compile the oracle's C sources with gcc -O2 into oracle/liboracle.so."""
    if force or _stale():
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _stale():
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    graph_args = [ctypes.c_int, P, ctypes.c_int, P, P, P]
    lib.oracle_kbest.argtypes = graph_args + graph_args + [P, i64, P, P]
    lib.oracle_kbest.restype = ctypes.c_int
    lib.oracle_kbest_ex.argtypes = graph_args + graph_args + [P, i64, ctypes.c_int, ctypes.c_int, P, P]
    lib.oracle_kbest_ex.restype = ctypes.c_int
    lib.oracle_exact.argtypes = graph_args + graph_args + [P, ctypes.c_int, ctypes.c_double, P, P]
    lib.oracle_exact.restype = ctypes.c_int
    lib.oracle_induced_cost.argtypes = graph_args + graph_args + [P, ctypes.c_int, P, P]
    lib.oracle_induced_cost.restype = ctypes.c_int
    lib.oracle_count_mappings.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_count_mappings.restype = ctypes.c_double
    lib.oracle_kbest_cand.argtypes = graph_args + graph_args + [P, i64, ctypes.c_int, ctypes.c_int, P, P, P]
    lib.oracle_kbest_cand.restype = ctypes.c_int
    lib.oracle_kbest_pairs.argtypes = [P] * 9 + [i64, P, i64, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_kbest_pairs.restype = ctypes.c_int
    lib.oracle_bipartite.argtypes = graph_args + graph_args + [P, i64, P, P, P, P, P, P, P]
    lib.oracle_bipartite.restype = ctypes.c_int
    lib.oracle_bipartite_pairs.argtypes = [P] * 9 + [i64, P, i64, P, P, P, P, P, P]
    lib.oracle_bipartite_pairs.restype = ctypes.c_int
    _lib = lib
    return lib


def _arr(a, dt=np.int32) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_args(g, keep: list):
    vl = _arr(g.vlabel)
    eu = _arr(g.eu)
    ev = _arr(g.ev)
    el = None if getattr(g, "elabel", None) is None else _arr(g.elabel)
    keep += [vl, eu, ev, el]
    return [int(g.n), _ptr(vl), int(eu.shape[0]), _ptr(eu), _ptr(ev), _ptr(el)]


def _check(st: int, what: str):
    if st != OR_OK:
        raise OracleError(f"{what}: oracle status {st}")


def kbest(g1, g2, costs: Sequence[int], K: int, last_complete: bool = False,
          directed: bool = False, with_cand: bool = False):
    """K-Best search g1 -> g2; returns (distance, mapping) with -1 = deleted,
    and with with_cand also the number of children generated over all levels.

    last_complete: complete every child of the last level and keep the least total
    (instead of keeping the K of least partial distance, then completing).
    directed: edge k is the arc eu[k] -> ev[k]; each arc is one edit operation."""
    lib = _load()
    keep: list = []
    c = _arr(costs)
    dist = ctypes.c_int64(0)
    cand = ctypes.c_int64(0)
    mp = np.zeros(max(int(g1.n), 1), dtype=np.int32)
    st = lib.oracle_kbest_cand(*_graph_args(g1, keep), *_graph_args(g2, keep), _ptr(c), int(K),
                               1 if last_complete else 0, 1 if directed else 0, ctypes.byref(dist), _ptr(mp),
                               ctypes.byref(cand))
    _check(st, "kbest")
    if with_cand:
        return int(dist.value), mp[: int(g1.n)].copy(), int(cand.value)
    return int(dist.value), mp[: int(g1.n)].copy()


def exact(g1, g2, costs: Sequence[int], max_mappings: float = 1e8,
          directed: bool = False) -> Tuple[int, np.ndarray]:
    """Exact GED by enumerating every injective partial mapping."""
    lib = _load()
    keep: list = []
    c = _arr(costs)
    dist = ctypes.c_int64(0)
    mp = np.zeros(max(int(g1.n), 1), dtype=np.int32)
    st = lib.oracle_exact(*_graph_args(g1, keep), *_graph_args(g2, keep), _ptr(c),
                          1 if directed else 0, float(max_mappings), ctypes.byref(dist), _ptr(mp))
    _check(st, "exact")
    return int(dist.value), mp[: int(g1.n)].copy()


def induced_cost(g1, g2, costs: Sequence[int], mapping, directed: bool = False) -> int:
    """Edit cost of a complete mapping (mapping[v] = -1 deletes v)."""
    lib = _load()
    keep: list = []
    c = _arr(costs)
    mp = _arr(mapping)
    if mp.shape[0] != int(g1.n):
        raise OracleError("mapping length must equal g1.n")
    out = ctypes.c_int64(0)
    st = lib.oracle_induced_cost(*_graph_args(g1, keep), *_graph_args(g2, keep), _ptr(c),
                                 1 if directed else 0, _ptr(mp if mp.size else np.zeros(1, np.int32)), ctypes.byref(out))
    _check(st, "induced_cost")
    return int(out.value)


def count_mappings(n1: int, n2: int) -> float:
    """Number of complete mappings g1 -> g2 (sum over s of C(n1,s) n2!/(n2-s)!)."""
    return float(_load().oracle_count_mappings(int(n1), int(n2)))


def map_offsets(graphs, pairs: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum of the source orders: where each pair's mapping starts."""
    n_src = np.asarray(graphs.n, dtype=np.int64)[np.asarray(pairs)[:, 0]]
    off = np.zeros(len(n_src), dtype=np.int64)
    if len(n_src) > 1:
        np.cumsum(n_src[:-1], out=off[1:])
    return off


def kbest_pairs(graphs, pairs: np.ndarray, costs: Sequence[int], K: int, last_complete: bool = False,
                directed: bool = False, with_cand: bool = False):
    """Run the oracle over many pairs of a GraphSet.

    Returns (dist int64 [P], maps int32 [sum n_src], offsets int64 [P]), and with
    with_cand also the children generated per pair (int64 [P]).
    """
    lib = _load()
    pairs = _arr(pairs, np.int64).reshape(-1, 2)
    off = map_offsets(graphs, pairs)
    total = int(np.asarray(graphs.n, np.int64)[pairs[:, 0]].sum()) if len(pairs) else 0
    dist = np.zeros(len(pairs), dtype=np.int64)
    maps = np.zeros(max(total, 1), dtype=np.int32)
    n = _arr(graphs.n)
    m = _arr(graphs.m)
    voff = _arr(graphs.voff, np.int64)
    eoff = _arr(graphs.eoff, np.int64)
    vl = _arr(graphs.vlabel) if len(graphs.vlabel) else np.zeros(1, np.int32)
    eu = _arr(graphs.eu) if len(graphs.eu) else np.zeros(1, np.int32)
    ev = _arr(graphs.ev) if len(graphs.ev) else np.zeros(1, np.int32)
    el = None if graphs.elabel is None else (_arr(graphs.elabel) if len(graphs.elabel) else np.zeros(1, np.int32))
    c = _arr(costs)
    cand = np.zeros(max(len(pairs), 1), dtype=np.int64)
    failed = ctypes.c_int64(-1)
    st = lib.oracle_kbest_pairs(_ptr(n), _ptr(m), _ptr(voff), _ptr(eoff), _ptr(vl), _ptr(eu),
                                _ptr(ev), _ptr(el), _ptr(pairs), int(len(pairs)), _ptr(c), int(K),
                                1 if last_complete else 0, 1 if directed else 0, _ptr(dist), _ptr(maps), _ptr(off),
                                _ptr(cand), ctypes.byref(failed))
    _check(st, f"kbest_pairs (pair {failed.value})")
    if with_cand:
        return dist, maps[:total], off, cand[:len(pairs)]
    return dist, maps[:total], off


def bipartite(g1, g2, costs: Sequence[int], K: int, trace: bool = False):
    """Bipartite K-best bound g1 -> g2: (distance, mapping, solves), and with
    trace=True also (assignment costs [npop], mappings [npop, n1]) of the popped
    assignments in pop order."""
    lib = _load()
    keep: list = []
    c = _arr(costs)
    dist = ctypes.c_int64(0)
    solves = ctypes.c_int64(0)
    n1 = int(g1.n)
    mp = np.zeros(max(n1, 1), dtype=np.int32)
    pc = pm = None
    npop = ctypes.c_int64(0)
    if trace:
        pc = np.zeros(max(int(K), 1), dtype=np.int64)
        pm = np.zeros(max(int(K) * n1, 1), dtype=np.int32)
    st = lib.oracle_bipartite(*_graph_args(g1, keep), *_graph_args(g2, keep), _ptr(c), int(K),
                              ctypes.byref(dist), _ptr(mp), ctypes.byref(solves), _ptr(pc), _ptr(pm),
                              ctypes.byref(npop), None)
    _check(st, "bipartite")
    out = (int(dist.value), mp[:n1].copy(), int(solves.value))
    if trace:
        k = int(npop.value)
        return out + (pc[:k].copy(), pm[:k * n1].reshape(k, n1).copy())
    return out


def bipartite_pairs(graphs, pairs: np.ndarray, costs: Sequence[int], K: int, with_steps: bool = False):
    """bipartite() over many pairs of a GraphSet: (dist int64 [P], maps int32
    [sum n_src], offsets int64 [P], solves int64 [P]), and with with_steps the
    solver's search steps per pair (each relaxes every column from one row)."""
    lib = _load()
    pairs = _arr(pairs, np.int64).reshape(-1, 2)
    off = map_offsets(graphs, pairs)
    total = int(np.asarray(graphs.n, np.int64)[pairs[:, 0]].sum()) if len(pairs) else 0
    dist = np.zeros(len(pairs), dtype=np.int64)
    solves = np.zeros(len(pairs), dtype=np.int64)
    steps = np.zeros(len(pairs), dtype=np.int64)
    maps = np.zeros(max(total, 1), dtype=np.int32)
    n = _arr(graphs.n)
    m = _arr(graphs.m)
    voff = _arr(graphs.voff, np.int64)
    eoff = _arr(graphs.eoff, np.int64)
    vl = _arr(graphs.vlabel) if len(graphs.vlabel) else np.zeros(1, np.int32)
    eu = _arr(graphs.eu) if len(graphs.eu) else np.zeros(1, np.int32)
    ev = _arr(graphs.ev) if len(graphs.ev) else np.zeros(1, np.int32)
    el = None if graphs.elabel is None else (_arr(graphs.elabel) if len(graphs.elabel) else np.zeros(1, np.int32))
    c = _arr(costs)
    failed = ctypes.c_int64(-1)
    st = lib.oracle_bipartite_pairs(_ptr(n), _ptr(m), _ptr(voff), _ptr(eoff), _ptr(vl), _ptr(eu),
                                    _ptr(ev), _ptr(el), _ptr(pairs), int(len(pairs)), _ptr(c), int(K),
                                    _ptr(dist), _ptr(maps), _ptr(off), _ptr(solves), _ptr(steps),
                                    ctypes.byref(failed))
    _check(st, f"bipartite_pairs (pair {failed.value})")
    if with_steps:
        return dist, maps[:total], off, solves, steps
    return dist, maps[:total], off, solves


def edit_path(g1, g2, costs: Sequence[int], mapping, directed: bool = False):
    """The explicit edit operations of a complete mapping (Sec. 2.2-2.4), plain
    Python: list of (kind, a, b, c, d, cost) with kind 0..5 = vertex substitution,
    vertex deletion, vertex insertion, edge substitution, edge deletion, edge
    insertion, in the order: g1 vertices ascending (substituted or deleted),
    inserted g2 vertices ascending, g1 edges (a < b) lexicographically
    (substituted onto a g2 edge, or deleted), uncovered g2 edges (c < d)
    lexicographically (inserted).  The costs sum to the mapping's edit cost.
    directed: edges are arcs (a, b), listed in lexicographic order of (a, b); a
    substituted arc's image is (phi(a), phi(b)) as it stands."""
    vsub, vdel, vins, esub, edel, eins = (int(x) for x in costs)
    n1, n2 = int(g1.n), int(g2.n)
    phi = [int(x) for x in mapping]

    def key(a, b):
        return (a, b) if directed else (min(a, b), max(a, b))

    def edges(g):
        el = g.elabel if getattr(g, "elabel", None) is not None else [0] * len(g.eu)
        return {key(int(a), int(b)): int(l) for a, b, l in zip(g.eu, g.ev, el)}

    E1, E2 = edges(g1), edges(g2)
    pre = {}
    for v in range(n1):
        if phi[v] >= 0:
            pre[phi[v]] = v
    ops = []
    for v in range(n1):
        u = phi[v]
        if u >= 0:
            ops.append((0, v, u, -1, -1, vsub if int(g1.vlabel[v]) != int(g2.vlabel[u]) else 0))
        else:
            ops.append((1, v, -1, -1, -1, vdel))
    for u in range(n2):
        if u not in pre:
            ops.append((2, -1, u, -1, -1, vins))
    for (a, b) in sorted(E1):
        x, y = phi[a], phi[b]
        img = key(x, y)
        if x >= 0 and y >= 0 and img in E2:
            ops.append((3, a, b, img[0], img[1], esub if E1[(a, b)] != E2[img] else 0))
        else:
            ops.append((4, a, b, -1, -1, edel))
    for (c, d) in sorted(E2):
        a, b = pre.get(c, -1), pre.get(d, -1)
        if not (a >= 0 and b >= 0 and key(a, b) in E1):
            ops.append((5, -1, -1, c, d, eins))
    return ops
