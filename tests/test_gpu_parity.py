"""GPU parity: distances and mappings from libged equal the CPU oracle's
bit for bit on the same seeded inputs (run on an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import Graph, GraphSet

pytestmark = pytest.mark.gpu

UNIT = synth.UNIT_COSTS
PAPER = synth.PAPER_COSTS
HIGH = (4, 12, 12, 1, 10, 10)
ODD = (3, 1, 2, 5, 1, 3)


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


SCHEDULES = [0, 1]   # library's choice (wavefront kernel where eligible), workgroup kernel only


def gpu_vs_oracle(ged, graphs, pairs, costs, K, perpair=False, db=None, schedule=0):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    say(f"  case: {len(pairs)} pairs, K={K}, costs={costs}, perpair={perpair}, schedule={schedule}")
    own = db is None
    if own:
        db = ged.Database(graphs)
    res = ged.kbest(db, pairs, costs, K, perpair=perpair, with_cand=True, schedule=schedule)
    if own:
        db.close()
    d, m, off, cand = oracle.kbest_pairs(graphs, pairs, costs, K, with_cand=True)
    np.testing.assert_array_equal(res.offsets, off)
    bad = np.nonzero(res.dist != d)[0]
    assert bad.size == 0, f"dist differs on pairs {bad[:10].tolist()}: gpu {res.dist[bad[:10]].tolist()} oracle {d[bad[:10]].tolist()}"
    np.testing.assert_array_equal(res.maps, m)
    # the children whose partial edit distance the search evaluated: the
    # oracle's count of generated children (Sec. 4.2.1 branching), per pair
    np.testing.assert_array_equal(res.cand, cand)
    return res


def tiny_set(seed, count, n_max, p, nvl, nel):
    gs = [synth.random_small_graph(seed, k, n_max, p, nvl, nel) for k in range(count)]
    return GraphSet.from_graphs(gs)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("costs", [UNIT, PAPER, ODD, HIGH])
@pytest.mark.parametrize("K", [1, 2, 3, 7, 63, 64, 65, 128, 1024])
def test_tiny_random_pairs(ged, costs, K, schedule):
    graphs = tiny_set(100 + K, 60, 9, 0.45, 3, 3)
    pairs = [[2 * k, 2 * k + 1] for k in range(30)] + [[k, k] for k in range(0, 60, 7)]
    gpu_vs_oracle(ged, graphs, pairs, costs, K, schedule=schedule)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("costs", [
    (40, 90, 70, 25, 60, 45),        # thresholds near 127 above the least child: both counting paths
    (1000, 3000, 2500, 700, 1300, 900),  # thresholds far above it: full-width counts every level
    (4_194_304, 5_000_011, 4_500_007, 4_300_003, 4_200_001, 4_250_017),  # a cost >= 2^22: 32-bit products
])
@pytest.mark.parametrize("K", [16, 64])
def test_cost_scales(ged, costs, K, schedule):
    """Small pairs (the wavefront kernel's range) under cost scales that move the K-th
    smallest PED in and out of the byte-packed window, and past 24-bit products."""
    gs = []
    for k in range(36):
        g = synth.er_graph(61, k, 10, 24, 0.1, 0.3, 4)
        if k % 3 == 0:
            g.elabel = (np.arange(g.m) % 3).astype(np.int32)
        gs.append(g)
    graphs = GraphSet.from_graphs(gs)
    pairs = [[2 * k, 2 * k + 1] for k in range(18)] + [[k, (k * 7 + 3) % 36] for k in range(18)]
    gpu_vs_oracle(ged, graphs, pairs, costs, K, schedule=schedule)


def test_identity_is_zero(ged):
    graphs = tiny_set(7, 20, 12, 0.4, 4, 2)
    pairs = [[k, k] for k in range(20)]
    res = gpu_vs_oracle(ged, graphs, pairs, PAPER, 3)
    assert (res.dist == 0).all()


def test_empty_graphs(ged):
    z = np.zeros(0, np.int32)
    empty = Graph(0, z, z, z, z)
    g = synth.random_small_graph(9, 0, 7, 0.5, 3, 2, n_min=5)
    graphs = GraphSet.from_graphs([empty, g, empty])
    pairs = [[0, 1], [1, 0], [0, 2], [1, 1]]
    for costs in (UNIT, PAPER, ODD):
        res = gpu_vs_oracle(ged, graphs, pairs, costs, 4)
        assert res.dist[0] == costs[2] * g.n + costs[5] * g.m
        assert res.dist[1] == costs[1] * g.n + costs[4] * g.m
        assert res.dist[2] == 0


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("K", [1, 16, 64, 1024])
def test_pair_er_8x9(ged, K, schedule):
    w = synth.pair_er_8x9()
    gpu_vs_oracle(ged, w.graphs, [[0, 1], [1, 0]], w.costs, K, schedule=schedule)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_batch_er_subset(ged, schedule):
    w = synth.batch_er_10_30(512)
    gpu_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K, schedule=schedule)


@pytest.mark.parametrize("K", [5, 32, 64])
def test_wave_size_limits(ged, K):
    """Pairs at and around the wavefront kernel's limits (n = 31, 32, 33), labelled edges,
    dense and empty graphs, run in one batch so both kernels share a launch plan."""
    gs = []
    for k, (n, p) in enumerate([(32, 0.5), (32, 0.0), (31, 0.9), (33, 0.3), (1, 0.0), (32, 1.0),
                                (20, 0.3), (32, 0.25)]):
        g = synth.er_graph(23, k, n, n, p, p, 4)
        g.elabel = (np.arange(g.m) % 5).astype(np.int32)
        gs.append(g)
    graphs = GraphSet.from_graphs(gs)
    pairs = [[a, b] for a in range(len(gs)) for b in range(len(gs))]
    for costs in (UNIT, ODD):
        res = gpu_vs_oracle(ged, graphs, pairs, costs, K, schedule=0)
        res2 = gpu_vs_oracle(ged, graphs, pairs, costs, K, schedule=1)
        np.testing.assert_array_equal(res.cand, res2.cand)


# the last: vertex costs >= 2^22 (32-bit products); edge costs stay small enough that
# the complete 64-vertex graph cannot overflow int32
WAVE64_COSTS = [UNIT, ODD, (40, 90, 70, 25, 60, 45), (1000, 3000, 2500, 700, 1300, 900),
                (4_194_304, 5_000_011, 4_500_007, 30_011, 20_021, 35_003)]


def wave64_set():
    """1..64 vertices: both word boundaries, empty and complete graphs, labelled edges."""
    gs = []
    for k, (n, p) in enumerate([(64, 0.1), (64, 0.0), (63, 0.3), (33, 0.2), (48, 0.05), (64, 1.0),
                                (40, 0.15), (57, 0.08), (20, 0.3), (35, 0.5), (1, 0.0)]):
        g = synth.er_graph(29, k, n, n, p, p, 4)
        if k % 2 == 0:
            g.elabel = (np.arange(g.m) % 5).astype(np.int32)
        gs.append(g)
    return GraphSet.from_graphs(gs)


@pytest.mark.parametrize("costs", WAVE64_COSTS)
@pytest.mark.parametrize("K", [1, 3, 16, 63, 64])
def test_wave64_range(ged, costs, K):
    """Pairs of 33..64 vertices (the two-word wavefront kernel): both word boundaries,
    empty and complete graphs, labelled edges, cost scales that put the K-th smallest
    child inside the first byte window, past it (bucket passes) and past 24-bit
    products.  The workgroup kernel must agree on the candidate counts as well."""
    graphs = wave64_set()
    n = graphs.n
    pairs = [[a, b] for a in range(len(n)) for b in range(len(n)) if max(n[a], n[b]) > 32]
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K)
    kinds = {name for name, *_ in plan.bins()}
    plan.close()
    assert kinds == {"kb_wave2_kernel"}, kinds
    res = gpu_vs_oracle(ged, graphs, pairs, costs, K, db=db, schedule=0)
    res2 = ged.kbest(db, pairs, costs, K, with_cand=True, schedule=1)
    db.close()
    np.testing.assert_array_equal(res.dist, res2.dist)
    np.testing.assert_array_equal(res.maps, res2.maps)
    np.testing.assert_array_equal(res.cand, res2.cand)


@pytest.mark.parametrize("costs", WAVE64_COSTS)
@pytest.mark.parametrize("K", [65, 100, 128])
def test_wave64_two_slots(ged, costs, K):
    """Beams of 65..128 slots (two slots per lane of the two-word wavefront kernel) on
    every pair of 1..64 vertices, the ones of up to 32 included: the same cost scales
    (byte window, bucket passes, 32-bit products); the workgroup kernel agrees on
    distances, mappings and candidate counts."""
    graphs = wave64_set()
    nn = len(graphs.n)
    pairs = [[a, b] for a in range(nn) for b in range(nn)]
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K)
    kinds = {name for name, *_ in plan.bins()}
    plan.close()
    assert kinds == {"kb_wave2_kernel"}, kinds
    res = gpu_vs_oracle(ged, graphs, pairs, costs, K, db=db, schedule=0)
    res2 = ged.kbest(db, pairs, costs, K, with_cand=True, schedule=1)
    db.close()
    np.testing.assert_array_equal(res.dist, res2.dist)
    np.testing.assert_array_equal(res.maps, res2.maps)
    np.testing.assert_array_equal(res.cand, res2.cand)


def wide_source_set():
    """Sources of 65..128 vertices and targets of 0..64 (both ends of each range, empty
    and edgeless graphs, labelled edges); returns the set and the number of sources."""
    z = np.zeros(0, np.int32)
    src = [(128, 0.05), (65, 0.1), (100, 0.03), (128, 0.0), (90, 0.08), (70, 0.2)]
    dst = [(64, 0.1), (1, 0.0), (33, 0.2), (64, 0.0), (20, 0.3), (0, 0.0), (48, 0.06)]
    gs = []
    for k, (n, p) in enumerate(src + dst):
        if n == 0:
            gs.append(Graph(0, z, z, z, z))
            continue
        g = synth.er_graph(37, k, n, n, p, p, 4)
        if k % 2 == 1:
            g.elabel = (np.arange(g.m) % 5).astype(np.int32)
        gs.append(g)
    return GraphSet.from_graphs(gs), len(src)


@pytest.mark.parametrize("costs", WAVE64_COSTS[:4])
@pytest.mark.parametrize("K", [1, 16, 64, 128])
def test_wide_source_wave(ged, costs, K):
    """Sources of 65..128 vertices against targets of up to 64: the two-word wavefront
    kernel with a 128-vertex mapping (one beam slot per lane up to K = 64, two above);
    the workgroup kernel agrees on distances, mappings and candidate counts."""
    graphs, ns = wide_source_set()
    pairs = [[a, ns + b] for a in range(ns) for b in range(len(graphs.n) - ns)]
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K)
    kinds = {name for name, *_ in plan.bins()}
    plan.close()
    assert kinds == {"kb_wave2_kernel"}, kinds
    res = gpu_vs_oracle(ged, graphs, pairs, costs, K, db=db, schedule=0)
    res2 = ged.kbest(db, pairs, costs, K, with_cand=True, schedule=1)
    db.close()
    np.testing.assert_array_equal(res.dist, res2.dist)
    np.testing.assert_array_equal(res.maps, res2.maps)
    np.testing.assert_array_equal(res.cand, res2.cand)


@pytest.mark.parametrize("K", [8, 64, 128])
def test_query_molecule_wave64(ged, K):
    """Molecule-like pairs (n 10..70): the wavefront bins (n <= 32 and n <= 64 at K <= 64,
    the two-slot one for n <= 64 at K = 128, sources above 64 against targets of up to
    64) and the workgroup bin for targets above 64 in one plan."""
    w = synth.query_molecule_10_70(200)
    gpu_vs_oracle(ged, w.graphs, w.pairs, w.costs, K)


def test_query_molecule_subset(ged):
    w = synth.query_molecule_10_70(120)
    gpu_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K)


def test_stress_smallest_pairs(ged):
    w = synth.stress_er_100_500(256)
    size = w.graphs.n[w.pairs].max(1)
    pick = w.pairs[np.argsort(size, kind="stable")[:2]]
    gpu_vs_oracle(ged, w.graphs, pick, w.costs, w.K)


@pytest.mark.parametrize("n1,n2", [(33, 31), (31, 33), (64, 65), (65, 64), (40, 100), (100, 40),
                                   (130, 129), (300, 260)])
def test_word_boundaries(ged, n1, n2):
    g1 = synth.er_graph(13, n1, n1, n1, 0.2, 0.2, 3)
    g2 = synth.er_graph(14, n2, n2, n2, 0.2, 0.2, 3)
    graphs = GraphSet.from_graphs([g1, g2])
    gpu_vs_oracle(ged, graphs, [[0, 1], [1, 0]], UNIT, 8)


def test_max_order(ged):
    g1 = synth.er_graph(15, 0, 512, 512, 0.3, 0.3, 4)
    g2 = synth.er_graph(15, 1, 512, 512, 0.3, 0.3, 4)
    graphs = GraphSet.from_graphs([g1, g2])
    gpu_vs_oracle(ged, graphs, [[0, 1]], UNIT, 4)


def test_labelled_edges_many_planes(ged):
    gs = [synth.random_small_graph(17, k, 20, 0.4, 3, 16, n_min=10) for k in range(16)]
    graphs = GraphSet.from_graphs(gs)
    pairs = [[2 * k, 2 * k + 1] for k in range(8)]
    gpu_vs_oracle(ged, graphs, pairs, PAPER, 32)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_perpair_equals_batched(ged, schedule):
    w = synth.batch_er_10_30(96)
    res = gpu_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K, perpair=True, schedule=schedule)
    db = ged.Database(w.graphs)
    res2 = ged.kbest(db, w.pairs, w.costs, w.K, with_cand=True)
    db.close()
    np.testing.assert_array_equal(res.dist, res2.dist)
    np.testing.assert_array_equal(res.maps, res2.maps)
    np.testing.assert_array_equal(res.cand, res2.cand)


def test_repeat_runs_identical(ged):
    w = synth.batch_er_10_30(256)
    db = ged.Database(w.graphs)
    plan = ged.Plan(db, w.pairs, w.K)
    outs = []
    for _ in range(3):
        dist, maps, cand = plan.outputs(with_cand=True)
        plan.run(w.costs, dist, maps, cand)
        outs.append((dist.cpu().numpy(), maps.cpu().numpy(), cand.cpu().numpy()))
    plan.close()
    db.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)


def test_errors(ged):
    w = synth.pair_er_8x9()
    db = ged.Database(w.graphs)
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[0, 1]], 0)
    assert e.value.status == ged.GED_EINVAL
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[0, 1]], ged.MAX_K + 1)
    assert e.value.status == ged.GED_EUNSUPPORTED
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[0, 2]], 4)
    assert e.value.status == ged.GED_EINVAL
    plan = ged.Plan(db, [[0, 1]], 4)
    dist, maps, _ = plan.outputs()
    with pytest.raises(ged.GedError) as e:
        plan.run((1, -1, 1, 1, 1, 1), dist, maps)
    assert e.value.status == ged.GED_EINVAL
    with pytest.raises(ged.GedError) as e:
        plan.run((2 ** 30, 1, 1, 1, 1, 1), dist, maps)
    assert e.value.status == ged.GED_EINVAL and "overflow" in str(e.value)
    plan.close()
    empty = ged.Plan(db, np.zeros((0, 2), np.int64), 4)
    d0, m0, _ = empty.outputs()
    empty.run(UNIT, d0, m0)
    empty.close()
    db.close()
