"""Edit-path output (ged_edit_path, kb_path_kernel) against the oracle's
expansion, operation for operation, on mappings returned by the tree search and
the bipartite method: small and 512-vertex pairs, no / two / four edge-label
planes, empty graphs; the costs of each pair sum to the distance the search
returned; invalid mappings are rejected (GPU)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import GraphSet

pytestmark = pytest.mark.gpu

PAPER = synth.PAPER_COSTS
NONMETRIC = (3, 2, 5, 9, 1, 2)


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


def check_paths(ged, graphs, pairs, costs, K, method=0):
    import torch
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    say(f"  case: {len(pairs)} pairs, K={K}, costs={costs}, method={method}")
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K, method=method)
    dist, maps, _ = plan.outputs()
    plan.run(costs, dist, maps)
    torch.cuda.synchronize()
    ops, off, cnt = ged.edit_path(db, pairs, costs, maps)
    d = dist[:len(pairs)].cpu().numpy()
    m = maps[:plan.map_size].cpu().numpy()
    plan.close()
    db.close()
    n = graphs.n
    moff = np.concatenate([[0], np.cumsum(n[pairs[:, 0]])])
    for q, (a, b) in enumerate(pairs):
        g1, g2 = graphs.graph(int(a)), graphs.graph(int(b))
        ref = oracle.edit_path(g1, g2, costs, m[moff[q]:moff[q + 1]])
        got = ops[off[q]:off[q] + cnt[q]]
        assert cnt[q] == len(ref), f"pair {q}: {cnt[q]} operations, oracle {len(ref)}"
        np.testing.assert_array_equal(got, np.asarray(ref, dtype=np.int32).reshape(-1, 6))
        assert int(got[:, 5].sum()) == d[q]
        assert cnt[q] <= off[q + 1] - off[q]


@pytest.mark.parametrize("costs", [synth.UNIT_COSTS, PAPER, NONMETRIC])
def test_tiny_pairs_tree_and_bipartite(ged, costs):
    gs = [synth.random_small_graph(107, k, 10, 0.45, 3, 4) for k in range(24)]
    graphs = GraphSet.from_graphs(gs)
    rng = np.random.default_rng(109)
    pairs = rng.integers(0, 24, size=(120, 2))
    check_paths(ged, graphs, pairs, costs, 8)
    check_paths(ged, graphs, pairs, costs, 8, method=1)


def test_batch_subset(ged):
    w = synth.batch_er_10_30(512)
    check_paths(ged, w.graphs, w.pairs, w.costs, w.K)


def test_molecule_labels(ged):
    w = synth.query_molecule_10_70(200)
    check_paths(ged, w.graphs, w.pairs, w.costs, 16)


def test_label_planes_four(ged):
    gs = [synth.random_small_graph(113, k, 30, 0.3, 3, 12, n_min=5) for k in range(12)]
    graphs = GraphSet.from_graphs(gs)
    pairs = [[a, b] for a in range(12) for b in range(12) if a != b][:60]
    check_paths(ged, graphs, pairs, NONMETRIC, 4)


def test_large_and_empty(ged):
    """512-vertex graphs (16 row words, two vertices per thread), and empty ones."""
    gs = [synth.er_graph(127, 0, 512, 512, 0.05, 0.05, 4), synth.er_graph(127, 1, 500, 500, 0.05, 0.05, 4),
          synth.er_graph(127, 2, 0, 0, 0.0, 0.0, 2), synth.er_graph(127, 3, 7, 7, 0.5, 0.5, 2)]
    gs[0].elabel = (np.arange(gs[0].m) % 3).astype(np.int32)
    gs[1].elabel = (np.arange(gs[1].m) % 2).astype(np.int32)
    graphs = GraphSet.from_graphs(gs)
    check_paths(ged, graphs, [[0, 1], [1, 0], [2, 3], [3, 2], [2, 2], [3, 3]], PAPER, 2)


def test_invalid_mapping(ged):
    import torch
    gs = [synth.random_small_graph(131, k, 8, 0.5, 2, 1, n_min=4) for k in range(3)]
    graphs = GraphSet.from_graphs(gs)
    db = ged.Database(graphs)
    n0 = int(graphs.n[0])
    for bad in ([0] * n0, [int(graphs.n[1])] + [-1] * (n0 - 1), [-2] + [-1] * (n0 - 1)):
        maps = torch.tensor(bad, dtype=torch.int32, device="cuda")
        with pytest.raises(ged.GedError) as e:
            ged.edit_path(db, [[0, 1]], PAPER, maps)
        assert e.value.status == ged.GED_EINVAL
    maps = torch.tensor([-1] * n0, dtype=torch.int32, device="cuda")
    ops, off, cnt = ged.edit_path(db, [[0, 1]], PAPER, maps)
    g1, g2 = graphs.graph(0), graphs.graph(1)
    assert cnt[0] == len(oracle.edit_path(g1, g2, PAPER, [-1] * n0))
    db.close()
