"""The bipartite method (GED_METHOD_BIPARTITE, kb_bip_kernel) against the
bipartite oracle bit for bit: distance, mapping and the number of assignment
problems solved, on seeded pairs from one-vertex graphs to n1 + n2 = 256 (one to
four columns per lane) and K up to 256 (one, two and four queue slots per lane),
with and without edge labels, at cost scales up to the solver's int32 bound (GPU)."""
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
NONMETRIC = (3, 2, 5, 9, 1, 2)
ODD = (3, 1, 2, 5, 1, 3)
LARGE = (700, 900, 1100, 300, 500, 400)


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


def bip_vs_oracle(ged, graphs, pairs, costs, K, db=None, perpair=False):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    say(f"  case: {len(pairs)} pairs, K={K}, costs={costs}, perpair={perpair}")
    own = db is None
    if own:
        db = ged.Database(graphs)
    res = ged.kbest(db, pairs, costs, K, with_cand=True, perpair=perpair, method=ged.METHOD_BIPARTITE)
    if own:
        db.close()
    d, m, off, s = oracle.bipartite_pairs(graphs, pairs, costs, K)
    np.testing.assert_array_equal(res.offsets, off)
    bad = np.nonzero(res.dist != d)[0]
    assert bad.size == 0, f"dist differs on pairs {bad[:10].tolist()}: gpu {res.dist[bad[:10]].tolist()} oracle {d[bad[:10]].tolist()}"
    np.testing.assert_array_equal(res.maps, m)
    np.testing.assert_array_equal(res.cand, s)
    return res


def tiny_set(seed, count, n_max, p, nvl, nel):
    return GraphSet.from_graphs([synth.random_small_graph(seed, k, n_max, p, nvl, nel) for k in range(count)])


@pytest.mark.parametrize("costs", [UNIT, PAPER, HIGH, NONMETRIC, ODD])
@pytest.mark.parametrize("K", [1, 2, 7, 64])
def test_tiny_random_pairs(ged, costs, K):
    graphs = tiny_set(61, 24, 9, 0.45, 3, 1)
    rng = np.random.default_rng(67)
    bip_vs_oracle(ged, graphs, rng.integers(0, 24, size=(160, 2)), costs, K)


@pytest.mark.parametrize("nel", [3, 9])
@pytest.mark.parametrize("K", [3, 40])
def test_edge_labels(ged, nel, K):
    """Two and four label planes: the incident-edge label counts of the matrix and
    the relabelled edges of the induced cost."""
    graphs = tiny_set(71, 20, 14, 0.4, 3, nel)
    rng = np.random.default_rng(73)
    for costs in (UNIT, NONMETRIC, LARGE):
        bip_vs_oracle(ged, graphs, rng.integers(0, 20, size=(60, 2)), costs, K)


@pytest.mark.parametrize("K", [1, 16, 64])
def test_order_limits(ged, K):
    """n1 + n2 up to 64 (both splits), one side empty, dense and empty graphs."""
    specs = [(32, 0.3), (32, 0.1), (63, 0.05), (1, 0.0), (0, 0.0), (64, 0.08), (40, 0.2), (24, 0.5),
             (31, 1.0), (33, 0.0)]
    gs = []
    for k, (n, p) in enumerate(specs):
        g = synth.er_graph(79, k, n, n, p, p, 4)
        if k % 3 == 0:
            g.elabel = (np.arange(g.m) % 3).astype(np.int32)
        gs.append(g)
    graphs = GraphSet.from_graphs(gs)
    n = graphs.n
    pairs = [[a, b] for a in range(len(gs)) for b in range(len(gs)) if n[a] + n[b] <= 64]
    bip_vs_oracle(ged, graphs, pairs, PAPER, K)


LARGE_SPECS = [(100, 0.05), (90, 0.08), (40, 0.2), (150, 0.03), (120, 0.04), (33, 0.3), (66, 0.1), (128, 0.02)]


def large_set():
    gs = []
    for k, (n, p) in enumerate(LARGE_SPECS):
        g = synth.er_graph(89, k, n, n, p, p, 4)
        if k % 2 == 0:
            g.elabel = (np.arange(g.m) % 3).astype(np.int32)
        gs.append(g)
    return GraphSet.from_graphs(gs)


@pytest.mark.parametrize("K", [8, 100])
def test_orders_past_64(ged, K):
    """n1 + n2 from 66 to 256: two, three and four columns per lane, labelled and
    unlabelled graphs, one and two queue slots per lane."""
    graphs = large_set()
    n = graphs.n
    pairs = [[a, b] for a in range(len(n)) for b in range(len(n)) if 64 < n[a] + n[b] <= 256]
    pick = pairs[1::4] if K == 100 else pairs[::2]
    m = np.asarray(n)[np.asarray(pick)].sum(1)
    assert len(set(((m + 63) // 64).tolist())) >= 3   # three column counts per lane
    bip_vs_oracle(ged, graphs, pick, PAPER, K)


def test_k256(ged):
    """Four queue slots per lane, across column counts."""
    graphs = large_set()
    bip_vs_oracle(ged, graphs, [[2, 5], [6, 2], [0, 2], [4, 6], [1, 5], [7, 6]], UNIT, 256)


def test_query_molecule_k128(ged):
    """The molecule query workload's shape at its K = 128 (n 10..70, three edge labels)."""
    w = synth.query_molecule_10_70(40)
    bip_vs_oracle(ged, w.graphs, w.pairs, w.costs, 128)


def test_pair_er_8x9(ged):
    w = synth.pair_er_8x9()
    bip_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K)


def test_batch_er_subset(ged):
    """The 4096-pair batch's first 384 pairs at K = 64."""
    w = synth.batch_er_10_30(384)
    bip_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K)


def test_perpair_and_tuned_equal(ged):
    w = synth.batch_er_10_30(96)
    db = ged.Database(w.graphs)
    ref = bip_vs_oracle(ged, w.graphs, w.pairs, w.costs, w.K, db=db)
    pp = ged.kbest(db, w.pairs, w.costs, w.K, with_cand=True, perpair=True, method=ged.METHOD_BIPARTITE)
    np.testing.assert_array_equal(pp.dist, ref.dist)
    np.testing.assert_array_equal(pp.maps, ref.maps)
    plan = ged.Plan(db, w.pairs, w.K, method=ged.METHOD_BIPARTITE)
    assert [b[0] for b in plan.bins()] == ["kb_bip_kernel"]
    dist, maps, cand = plan.outputs(with_cand=True)
    plan.tune(w.costs, dist, maps)
    for gpc in (1, 3):
        plan2 = ged.Plan(db, w.pairs, w.K, method=ged.METHOD_BIPARTITE, groups_per_cu=gpc)
        d2, m2, c2 = plan2.outputs(with_cand=True)
        plan2.run(w.costs, d2, m2, c2)
        import torch
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d2[:len(w.pairs)].cpu().numpy(), ref.dist)
        np.testing.assert_array_equal(m2[:plan2.map_size].cpu().numpy(), ref.maps)
        plan2.close()
    import torch
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dist[:len(w.pairs)].cpu().numpy(), ref.dist)
    plan.close()
    db.close()


def test_errors(ged):
    graphs = GraphSet.from_graphs([synth.er_graph(83, k, n, n, 0.02, 0.02, 3) for k, n in enumerate([140, 120, 5])])
    db = ged.Database(graphs)
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[0, 1]], 8, method=ged.METHOD_BIPARTITE)          # n1 + n2 = 260
    assert e.value.status == ged.GED_EUNSUPPORTED
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[2, 2]], 257, method=ged.METHOD_BIPARTITE)
    assert e.value.status == ged.GED_EUNSUPPORTED
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[2, 2]], 4, method=ged.METHOD_BIPARTITE, last_level=ged.LAST_COMPLETE)
    assert e.value.status == ged.GED_EINVAL
    with pytest.raises(ged.GedError) as e:
        ged.Plan(db, [[2, 2]], 4, method=7)
    assert e.value.status == ged.GED_EINVAL
    plan = ged.Plan(db, [[2, 1]], 4, method=ged.METHOD_BIPARTITE)
    dist, maps, cand = plan.outputs(with_cand=True)
    with pytest.raises(ged.GedError) as e:
        plan.run((1 << 18, 1, 1, 1, 1, 1), dist, maps, cand)            # past the solver's int32 bound
    assert e.value.status == ged.GED_EINVAL
    plan.close()
    db.close()
