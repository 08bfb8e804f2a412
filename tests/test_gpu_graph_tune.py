"""HIP-graph replay and the autotuner keep results bit-identical (GPU)."""
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


def mixed_workload():
    """Small ER and molecule-shaped pairs: a wavefront bin and workgroup bins (labelled edges)."""
    gs = [synth.er_graph(31, k, 10, 30, 0.1, 0.3, 5) for k in range(96)]
    gs += [synth.molecule_graph(32, k) for k in range(64)]
    graphs = GraphSet.from_graphs(gs)
    rng = np.random.default_rng(5)
    pairs = np.stack([rng.integers(0, len(gs), 200), rng.integers(0, len(gs), 200)], 1).astype(np.int64)
    return graphs, pairs


def test_graph_replay_matches_eager(ged):
    import torch
    graphs, pairs = mixed_workload()
    costs, K = synth.PAPER_COSTS, 48
    d_ref, m_ref, _ = oracle.kbest_pairs(graphs, pairs, costs, K)
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K)
    assert len(plan.bins()) >= 2
    other = ged.Plan(db, pairs[::-1].copy(), 7)
    od, om, _ = other.outputs()
    s = torch.cuda.Stream()
    dist, maps, cand = plan.outputs(with_cand=True)
    plan.capture(costs, dist, maps, cand, stream=s)
    # the null stream cannot be captured: rejected on the host before any HIP call
    st = ged.load().ged_plan_capture(plan._h, ged.Costs(*costs), dist.data_ptr(), maps.data_ptr(), None, None)
    assert st == ged.GED_EINVAL
    cands = []
    for rep in range(4):
        with torch.cuda.stream(s):
            dist.fill_(-7)
            maps.fill_(-7)
            cand.fill_(-7)
        plan.replay(stream=s)
        s.synchronize()
        np.testing.assert_array_equal(dist[:len(pairs)].cpu().numpy(), d_ref)
        np.testing.assert_array_equal(maps[:plan.map_size].cpu().numpy(), m_ref)
        cands.append(cand[:len(pairs)].cpu().numpy())
        # eager work of another plan between replays
        other.run(costs, od, om)
        torch.cuda.synchronize()
    for c in cands[1:]:
        np.testing.assert_array_equal(c, cands[0])
    plan.close()
    other.close()
    db.close()


def test_replay_without_capture_is_rejected(ged):
    w = synth.pair_er_8x9()
    db = ged.Database(w.graphs)
    plan = ged.Plan(db, w.pairs, 4)
    with pytest.raises(ged.GedError) as e:
        plan.replay()
    assert e.value.status == ged.GED_EINVAL
    plan.close()
    db.close()


def test_tune_keeps_results_and_caches(ged, tmp_path):
    graphs, pairs = mixed_workload()
    costs, K = synth.UNIT_COSTS, 64
    d_ref, m_ref, _ = oracle.kbest_pairs(graphs, pairs, costs, K)
    db = ged.Database(graphs)
    cache = str(tmp_path / "tune.txt")
    plan = ged.Plan(db, pairs, K)
    dist, maps, _ = plan.outputs()
    timed = plan.tune(costs, dist, maps, cache_path=cache)
    assert timed == len(plan.bins())
    np.testing.assert_array_equal(dist[:len(pairs)].cpu().numpy(), d_ref)
    np.testing.assert_array_equal(maps[:plan.map_size].cpu().numpy(), m_ref)
    chosen = plan.bins()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == len(chosen)

    plan2 = ged.Plan(db, pairs, K)
    d2, m2, _ = plan2.outputs()
    assert plan2.tune(costs, d2, m2, cache_path=cache) == 0
    assert plan2.bins() == chosen
    d2.fill_(0)
    plan2.run(costs, d2, m2)
    np.testing.assert_array_equal(d2[:len(pairs)].cpu().numpy(), d_ref)
    np.testing.assert_array_equal(m2[:plan2.map_size].cpu().numpy(), m_ref)
    plan.close()
    plan2.close()
    db.close()


@pytest.mark.parametrize("K", [64, 600])
def test_forced_workgroup_sizes_agree(ged, tmp_path, K):
    """The workgroup kernel at 256 and at 512 threads (and a one-workgroup-per-CU grid),
    forced through tuning-cache lines, gives the oracle's results; K = 600 makes the slot
    stride differ between the two sizes (768 and 1024)."""
    gs = [synth.random_small_graph(77, k, 12, 0.4, 3, 2) for k in range(40)]
    graphs = GraphSet.from_graphs(gs)
    pairs = np.array([[2 * k, 2 * k + 1] for k in range(20)], np.int64)
    costs = (2, 3, 3, 1, 2, 2)
    d_ref, m_ref, _ = oracle.kbest_pairs(graphs, pairs, costs, K)
    db = ged.Database(graphs)
    probe = str(tmp_path / "probe.txt")
    plan = ged.Plan(db, pairs, K, schedule=ged.SCHED_BLOCK)
    dist, maps, _ = plan.outputs()
    plan.tune(costs, dist, maps, cache_path=probe)
    keys = [line.split()[0] for line in open(probe).read().strip().splitlines()]
    assert keys
    plan.close()
    for threads in (256, 512):
        for gpc in (1, 2):
            forced = str(tmp_path / f"forced_{threads}_{gpc}.txt")
            with open(forced, "w") as f:
                for k in keys:
                    f.write(f"{k} 0 {gpc} {threads}\n")
            print(f"  case: K={K}, threads={threads}, groups_per_cu={gpc}", flush=True)
            p2 = ged.Plan(db, pairs, K, schedule=ged.SCHED_BLOCK)
            d2, m2, _ = p2.outputs()
            assert p2.tune(costs, d2, m2, cache_path=forced) == 0
            d2.fill_(-7)
            p2.run(costs, d2, m2)
            np.testing.assert_array_equal(d2[:len(pairs)].cpu().numpy(), d_ref)
            np.testing.assert_array_equal(m2[:p2.map_size].cpu().numpy(), m_ref)
            p2.close()
    db.close()


def test_bipartite_graph_replay_matches_eager(ged):
    """A bipartite plan with two bins (one and two columns per lane) captured once
    and replayed four times, with another plan's eager run between replays."""
    import torch
    gs = [synth.er_graph(33, k, 10, 30, 0.1, 0.3, 5) for k in range(40)]
    gs += [synth.er_graph(34, k, 40, 60, 0.05, 0.1, 5) for k in range(20)]
    graphs = GraphSet.from_graphs(gs)
    rng = np.random.default_rng(9)
    pairs = np.stack([rng.integers(0, len(gs), 120), rng.integers(0, len(gs), 120)], 1).astype(np.int64)
    costs, K = synth.PAPER_COSTS, 40
    d_ref, m_ref, _, s_ref = oracle.bipartite_pairs(graphs, pairs, costs, K)
    db = ged.Database(graphs)
    plan = ged.Plan(db, pairs, K, method=ged.METHOD_BIPARTITE)
    assert len(plan.bins()) == 2
    other = ged.Plan(db, pairs[::-1].copy(), 9, method=ged.METHOD_BIPARTITE)
    od, om, _ = other.outputs()
    s = torch.cuda.Stream()
    dist, maps, cand = plan.outputs(with_cand=True)
    plan.capture(costs, dist, maps, cand, stream=s)
    for rep in range(4):
        with torch.cuda.stream(s):
            dist.fill_(-7)
            maps.fill_(-7)
            cand.fill_(-7)
        plan.replay(stream=s)
        s.synchronize()
        np.testing.assert_array_equal(dist[:len(pairs)].cpu().numpy(), d_ref)
        np.testing.assert_array_equal(maps[:plan.map_size].cpu().numpy(), m_ref)
        np.testing.assert_array_equal(cand[:len(pairs)].cpu().numpy(), s_ref)
        other.run(costs, od, om)
        torch.cuda.synchronize()
    plan.close()
    other.close()
    db.close()
