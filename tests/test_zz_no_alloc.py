"""ged_kbest_noalloc (GPU): the allocation-free batched call against ged_kbest, its
allocating counterpart, on two calls in a row (the second on a smaller batch, so it
reuses the staging the first left behind), with pairs in every size bin of the
default schedule; a few pairs also against the oracle."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import GraphSet

pytestmark = pytest.mark.gpu


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


def mixed_set():
    """Graphs for every bin: n <= 32, <= 64, then 65..500 vertices (1..16 row words)."""
    gs = [synth.er_graph(151, k, 5, 32, 0.1, 0.3, 5) for k in range(40)]
    gs += [synth.er_graph(152, k, 33, 64, 0.05, 0.2, 5) for k in range(20)]
    gs += [synth.er_graph(153, k, 65, 500, 0.02, 0.1, 5) for k in range(16)]
    return GraphSet.from_graphs(gs)


def run_noalloc(ged, db, pairs, costs, K):
    import torch
    n_src = db.n[pairs[:, 0]].astype(np.int64)
    dist = torch.full((max(len(pairs), 1),), -7, dtype=torch.int32, device="cuda")
    maps = torch.full((max(int(n_src.sum()), 1),), -7, dtype=torch.int32, device="cuda")
    ged.kbest_noalloc(db, pairs, costs, K, dist, maps)
    return dist[:len(pairs)].cpu().numpy(), maps[:int(n_src.sum())].cpu().numpy()


@pytest.mark.parametrize("K,costs", [(16, synth.UNIT_COSTS), (64, synth.PAPER_COSTS), (128, synth.UNIT_COSTS)])
def test_noalloc_equals_kbest_twice(ged, K, costs):
    graphs = mixed_set()
    db = ged.Database(graphs)
    rng = np.random.default_rng(K)
    small = rng.integers(0, 40, size=(300, 2))
    mid = rng.integers(40, 60, size=(60, 2))
    big = np.stack([rng.integers(0, 76, 24), rng.integers(60, 76, 24)], 1)
    # sources of 65..128 vertices against targets of up to 64 (the third wavefront bin)
    n = graphs.n
    wsrc = [a for a in range(60, 76) if n[a] <= 128]
    assert wsrc, "the set has a source of 65..128 vertices"
    wide = np.stack([rng.choice(wsrc, 12), rng.integers(40, 60, 12)], 1)
    first = np.concatenate([small, mid, big, wide]).astype(np.int64)
    rng.shuffle(first)
    second = first[:97].copy()
    for name, pairs in (("first", first), ("second (smaller)", second)):
        say(f"  {name}: {len(pairs)} pairs, K={K}")
        d_na, m_na = run_noalloc(ged, db, pairs, costs, K)
        ref = ged.kbest(db, pairs, costs, K)
        np.testing.assert_array_equal(d_na, ref.dist)
        np.testing.assert_array_equal(m_na, ref.maps)
    # a few of the second call's pairs against the oracle as well
    sel = second[:6]
    d, m, off = oracle.kbest_pairs(graphs, sel, costs, K)
    np.testing.assert_array_equal(d_na[:6], d)
    np.testing.assert_array_equal(m_na[:int(graphs.n[sel[:, 0]].sum())], m)
    db.close()


def test_noalloc_directed(ged):
    gs = [synth.directed_graph(157, k, 5, 30, 0.05, 0.2, 3, 2) for k in range(20)]
    gs += [synth.directed_graph(158, k, 40, 120, 0.02, 0.05, 3, 2) for k in range(6)]
    graphs = GraphSet.from_graphs(gs)
    db = ged.Database(graphs, directed=True)
    rng = np.random.default_rng(5)
    pairs = rng.integers(0, 26, size=(120, 2)).astype(np.int64)
    for pp in (pairs, pairs[:31]):
        d_na, m_na = run_noalloc(ged, db, pp, synth.UNIT_COSTS, 32)
        ref = ged.kbest(db, pp, synth.UNIT_COSTS, 32)
        np.testing.assert_array_equal(d_na, ref.dist)
        np.testing.assert_array_equal(m_na, ref.maps)
    db.close()


def test_noalloc_errors(ged):
    import torch
    graphs = mixed_set()
    db = ged.Database(graphs)
    dist = torch.zeros(4, dtype=torch.int32, device="cuda")
    maps = torch.zeros(256, dtype=torch.int32, device="cuda")
    for pairs, K, costs, status in (([[0, 99]], 8, synth.UNIT_COSTS, ged.GED_EINVAL),
                                    ([[0, 1]], 0, synth.UNIT_COSTS, ged.GED_EINVAL),
                                    ([[0, 1]], 2000, synth.UNIT_COSTS, ged.GED_EUNSUPPORTED),
                                    ([[0, 1]], 8, (1, -1, 1, 1, 1, 1), ged.GED_EINVAL),
                                    ([[0, 1]], 8, (2**30, 2**30, 2**30, 1, 1, 1), ged.GED_EINVAL)):
        with pytest.raises(ged.GedError) as e:
            ged.kbest_noalloc(db, np.asarray(pairs, np.int64), costs, K, dist, maps)
        assert e.value.status == status
    # a batch whose staging exceeds the scratch: refused before anything runs
    many = np.zeros((2_000_000, 2), np.int64)
    with pytest.raises(ged.GedError) as e:
        ged.kbest_noalloc(db, many, synth.UNIT_COSTS, 8, dist, maps)
    assert e.value.status == ged.GED_EUNSUPPORTED and "scratch" in str(e.value)
    # an empty batch is a no-op
    ged.kbest_noalloc(db, np.zeros((0, 2), np.int64), synth.UNIT_COSTS, 8, dist, maps)
    db.close()
