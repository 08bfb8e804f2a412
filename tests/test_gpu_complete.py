"""Complete-then-minimum last level (GED_LAST_COMPLETE): every kernel family returns
the oracle's distance and mapping bit for bit; the candidate counts equal the default
search's (the same levels expand the same parents), and the distance is never above
the default search's, whose last-level children are a subset of those completed
here (GPU)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import GraphSet

pytestmark = pytest.mark.gpu

UNIT = synth.UNIT_COSTS
PAPER = synth.PAPER_COSTS
HIGH = (4, 12, 12, 1, 10, 10)
ODD = (3, 1, 2, 5, 1, 3)
WIDE_RANGE = (1000, 3000, 2500, 700, 1300, 900)
BIG_VERTEX = (4_194_304, 5_000_011, 4_500_007, 30_011, 20_021, 35_003)


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00830_amd import ged as g
    g.load()
    return g


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=0, db=None, kinds=None):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    say(f"  case: {len(pairs)} pairs, K={K}, costs={costs}, schedule={schedule}")
    own = db is None
    if own:
        db = ged.Database(graphs)
    if kinds is not None:
        plan = ged.Plan(db, pairs, K, schedule=schedule, last_level=ged.LAST_COMPLETE)
        got = {name for name, *_ in plan.bins()}
        plan.close()
        assert got == kinds, got
    res = ged.kbest(db, pairs, costs, K, with_cand=True, schedule=schedule, last_level=ged.LAST_COMPLETE)
    lit = ged.kbest(db, pairs, costs, K, with_cand=True, schedule=schedule)
    if own:
        db.close()
    d, m, off = oracle.kbest_pairs(graphs, pairs, costs, K, last_complete=True)
    np.testing.assert_array_equal(res.offsets, off)
    bad = np.nonzero(res.dist != d)[0]
    assert bad.size == 0, f"dist differs on pairs {bad[:10].tolist()}: gpu {res.dist[bad[:10]].tolist()} oracle {d[bad[:10]].tolist()}"
    np.testing.assert_array_equal(res.maps, m)
    np.testing.assert_array_equal(res.cand, lit.cand)
    assert (res.dist <= lit.dist).all()
    return res, lit


def tiny_set(seed, count, n_max, p, nvl, nel):
    gs = [synth.random_small_graph(seed, k, n_max, p, nvl, nel) for k in range(count)]
    return GraphSet.from_graphs(gs)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("costs", [UNIT, PAPER, ODD, HIGH])
@pytest.mark.parametrize("K", [1, 2, 7, 64, 65, 1024])
def test_tiny_random_pairs(ged, costs, K, schedule):
    graphs = tiny_set(41, 24, 9, 0.45, 3, 2)
    rng = np.random.default_rng(43)
    pairs = rng.integers(0, 24, size=(160, 2))
    complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=schedule)


def test_k1_is_greedy_and_beats_literal_somewhere(ged):
    """At K = 1 the default search keeps the least-PED child at the last level; the
    complete mode must find a strictly smaller distance on some pair of a random set
    (insertion costs differ by the last image), else the option changes nothing."""
    graphs = tiny_set(47, 30, 10, 0.5, 2, 1)
    rng = np.random.default_rng(53)
    pairs = rng.integers(0, 30, size=(300, 2))
    res, lit = complete_vs_oracle(ged, graphs, pairs, (1, 1, 5, 1, 1, 5), 1, schedule=0)
    assert (res.dist < lit.dist).any()


@pytest.mark.parametrize("K", [5, 64])
def test_wave_size_limits(ged, K):
    """n = 1, 20, 31, 32 and 33 with labelled edges, dense and empty graphs: the
    one-word wavefront kernel, the workgroup kernel, and both schedules in agreement."""
    gs = []
    for k, (n, p) in enumerate([(32, 0.5), (32, 0.0), (31, 0.9), (33, 0.3), (1, 0.0), (32, 1.0),
                                (20, 0.3), (32, 0.25)]):
        g = synth.er_graph(23, k, n, n, p, p, 4)
        g.elabel = (np.arange(g.m) % 5).astype(np.int32)
        gs.append(g)
    graphs = GraphSet.from_graphs(gs)
    pairs = [[a, b] for a in range(len(gs)) for b in range(len(gs))]
    for costs in (UNIT, ODD):
        r0, _ = complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=0)
        r1, _ = complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=1)
        np.testing.assert_array_equal(r0.cand, r1.cand)


WAVE64_COSTS = [UNIT, (40, 90, 70, 25, 60, 45), WIDE_RANGE, BIG_VERTEX]


@pytest.mark.parametrize("costs", WAVE64_COSTS)
@pytest.mark.parametrize("K", [1, 16, 64, 128])
def test_wave64_range(ged, costs, K):
    """Pairs of 33..64 vertices: the two-word wavefront kernel alone in the plan (two
    beam slots per lane at K = 128), then the workgroup kernel on the same pairs."""
    gs = []
    for k, (n, p) in enumerate([(64, 0.1), (64, 0.0), (63, 0.3), (33, 0.2), (48, 0.05), (64, 1.0),
                                (40, 0.15), (57, 0.08), (20, 0.3), (35, 0.5), (1, 0.0)]):
        g = synth.er_graph(29, k, n, n, p, p, 4)
        if k % 2 == 0:
            g.elabel = (np.arange(g.m) % 5).astype(np.int32)
        gs.append(g)
    graphs = GraphSet.from_graphs(gs)
    n = graphs.n
    pairs = [[a, b] for a in range(len(gs)) for b in range(len(gs)) if max(n[a], n[b]) > 32]
    db = ged.Database(graphs)
    complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=0, db=db, kinds={"kb_wave2_kernel"})
    complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=1, db=db)
    db.close()


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_er_subset(ged, schedule):
    w = synth.batch_er_10_30(256)
    complete_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K, schedule=schedule)


def test_query_molecule_subset(ged):
    """n 10..70 at K = 64: both wavefront bins and the workgroup bin in one plan."""
    w = synth.query_molecule_10_70(150)
    complete_vs_oracle(ged, w.graphs, w.pairs, w.costs, 64)


@pytest.mark.parametrize("K", [16, 128])
def test_wide_source_wave(ged, K):
    """Sources of 65..128 vertices against targets of up to 64 (the wavefront kernel's
    third family) with the last level completed, then the workgroup kernel."""
    from tests.test_gpu_parity import wide_source_set
    graphs, ns = wide_source_set()
    pairs = [[a, ns + b] for a in range(ns) for b in range(len(graphs.n) - ns)]
    db = ged.Database(graphs)
    for costs in (UNIT, WIDE_RANGE):
        complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=0, db=db, kinds={"kb_wave2_kernel"})
        complete_vs_oracle(ged, graphs, pairs, costs, K, schedule=1, db=db)
    db.close()


@pytest.mark.parametrize("n1,n2", [(64, 65), (65, 64), (40, 100), (130, 129)])
def test_word_boundaries(ged, n1, n2):
    g1 = synth.er_graph(13, n1, n1, n1, 0.2, 0.2, 3)
    g2 = synth.er_graph(14, n2, n2, n2, 0.2, 0.2, 3)
    graphs = GraphSet.from_graphs([g1, g2])
    complete_vs_oracle(ged, graphs, [[0, 1], [1, 0]], UNIT, 8)


def test_empty_graphs(ged):
    gs = [synth.er_graph(3, k, n, n, 0.3, 0.3, 2) for k, n in enumerate([0, 0, 1, 5])]
    graphs = GraphSet.from_graphs(gs)
    pairs = [[a, b] for a in range(4) for b in range(4)]
    for schedule in (0, 1):
        complete_vs_oracle(ged, graphs, pairs, PAPER, 4, schedule=schedule)


def labelled_set(seed, specs, nlab):
    gs = []
    for k, (n, p) in enumerate(specs):
        g = synth.er_graph(seed, k, n, n, p, p, 4)
        if nlab > 0:
            g.elabel = (np.arange(g.m) % nlab).astype(np.int32)
        gs.append(g)
    return GraphSet.from_graphs(gs)


@pytest.mark.parametrize("costs", [UNIT, PAPER, WIDE_RANGE, BIG_VERTEX])
@pytest.mark.parametrize("K", [1, 3, 64, 5000])
def test_wide_matches_oracle(ged, costs, K):
    """The single-pair search: empty and one-vertex graphs, 32-word boundaries,
    labelled edges, K from 1 to past the pair's level widths."""
    graphs = labelled_set(71, [(0, 0.0), (1, 0.0), (7, 0.5), (12, 0.3), (20, 0.2), (33, 0.1), (26, 0.6)], 3)
    db = ged.Database(graphs)
    pairs = [(2, 3), (3, 2), (4, 5), (5, 6), (6, 4), (0, 3), (3, 0), (1, 1)]
    d, m, off = oracle.kbest_pairs(graphs, np.asarray(pairs, np.int64), costs, K, last_complete=True)
    n = graphs.n
    for q, (a, b) in enumerate(pairs):
        say(f"  pair ({a},{b}) n1={n[a]} n2={n[b]} K={K} costs={costs}")
        dist, mp, cand = ged.kbest_wide(db, a, b, costs, K, last_level=ged.LAST_COMPLETE)
        assert dist == d[q], f"pair {q}: gpu {dist} oracle {d[q]}"
        np.testing.assert_array_equal(mp, m[off[q]:off[q] + n[a]])
        _, _, cand_lit = ged.kbest_wide(db, a, b, costs, K)
        assert cand == cand_lit
    db.close()


@pytest.mark.parametrize("K", [64, 1024])
def test_wide_equals_batched(ged, K):
    """Larger pairs (2, 4 and 10 target words): the single-pair search and the
    workgroup kernel agree in the complete mode too."""
    graphs = labelled_set(97, [(60, 0.1), (70, 0.08), (120, 0.04), (300, 0.02)], 3)
    db = ged.Database(graphs)
    pairs = [(0, 1), (1, 0), (2, 1), (1, 3)]
    ref = ged.kbest(db, pairs, PAPER, K, with_cand=True, schedule=1, last_level=ged.LAST_COMPLETE)
    for q, (a, b) in enumerate(pairs):
        say(f"  pair ({a},{b}) K={K}")
        dist, mp, cand = ged.kbest_wide(db, a, b, PAPER, K, last_level=ged.LAST_COMPLETE)
        assert dist == ref.dist[q]
        np.testing.assert_array_equal(mp, ref.mapping(q, graphs.n[a]))
        assert cand == ref.cand[q]
    db.close()


def test_wide_big_k_properties(ged):
    """K = 200,000 on a 100-vertex pair: an injective mapping whose induced cost
    (oracle) is the distance, never above the default search's."""
    graphs = labelled_set(101, [(100, 0.06), (100, 0.06)], 3)
    db = ged.Database(graphs)
    K = 200_000
    say(f"  pair (0,1) n=100 K={K}")
    d1, m1, c1 = ged.kbest_wide(db, 0, 1, PAPER, K, last_level=ged.LAST_COMPLETE)
    d0, _, c0 = ged.kbest_wide(db, 0, 1, PAPER, K)
    db.close()
    used = m1[m1 >= 0]
    assert len(np.unique(used)) == len(used) and (used < 100).all()
    assert oracle.induced_cost(graphs.graph(0), graphs.graph(1), PAPER, m1) == d1
    assert d1 <= d0 and c1 == c0


def test_bad_last_level(ged):
    graphs = tiny_set(59, 3, 6, 0.5, 2, 1)
    db = ged.Database(graphs)
    for bad in (-1, 2):
        with pytest.raises(ged.GedError) as e:
            ged.Plan(db, [[0, 1]], 4, last_level=bad)
        assert e.value.status == ged.GED_EINVAL
        with pytest.raises(ged.GedError) as e:
            ged.Wide(db, 0, 1, 4, last_level=bad)
        assert e.value.status == ged.GED_EINVAL
    db.close()
