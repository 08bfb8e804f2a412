"""Directed graphs (GED_DB_DIRECTED) through the two-word wavefront kernel
(pairs of up to 32 vertices, K <= 64) and the workgroup kernel (everything
else, and every pair under the workgroup-only schedule): distances and
mappings equal the oracle's directed search bit for bit, for every row width
(n up to 32, 64, 128, 256), no / two / four label planes (planes staged in
LDS and read from HBM), the candidate matrix in LDS and in the workspace,
256- and 512-thread workgroups, the complete-then-minimum last level and the
one-launch-per-pair path; the calls that take undirected graphs only refuse
a directed database (GPU)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import Graph, GraphSet

pytestmark = pytest.mark.gpu

UNIT = synth.UNIT_COSTS
PAPER = synth.PAPER_COSTS
NONMETRIC = (3, 2, 5, 9, 1, 2)
ASYM = (1, 1, 1, 7, 5, 3)


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


def directed_set(seed, count, n_lo, n_hi, p_lo, p_hi, nl=4, nel=0):
    return GraphSet.from_graphs([synth.directed_graph(seed, k, n_lo, n_hi, p_lo, p_hi, nl, nel)
                                 for k in range(count)])


def check(ged, graphs, pairs, costs, K, last_level=0, perpair=False, expect_words=None, schedule=0,
          kinds=None):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    say(f"  case: {len(pairs)} pairs, K={K}, costs={costs}, last={last_level}, perpair={perpair}, "
        f"schedule={schedule}, n<={int(graphs.n.max())}")
    db = ged.Database(graphs, directed=True)
    plan = ged.Plan(db, pairs, K, last_level=last_level, schedule=schedule)
    bins = plan.bins()
    names = {name for name, *_ in bins}
    assert names <= {"kb_block_kernel", "kb_wave2_kernel"}, bins
    if schedule == 1:
        assert names == {"kb_block_kernel"}, bins
    if kinds is not None:
        assert names == kinds, bins
    if expect_words is not None:
        assert {w for *_, w in bins} == expect_words, bins
    plan.close()
    res = ged.kbest(db, pairs, costs, K, perpair=perpair, last_level=last_level, schedule=schedule)
    db.close()
    d, m, off = oracle.kbest_pairs(graphs, pairs, costs, K, last_complete=last_level == 1, directed=True)
    np.testing.assert_array_equal(res.offsets, off)
    bad = np.nonzero(res.dist != d)[0]
    assert bad.size == 0, (f"dist differs on pairs {bad[:8].tolist()}: gpu {res.dist[bad[:8]].tolist()} "
                           f"oracle {d[bad[:8]].tolist()}")
    np.testing.assert_array_equal(res.maps, m)
    return res


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("costs", [UNIT, PAPER, NONMETRIC, ASYM])
@pytest.mark.parametrize("K", [1, 8, 64, 100])
def test_small_directed_pairs(ged, costs, K, schedule):
    """n 0..32 (two-word rows: out and in), unlabelled arcs, ragged orders incl. empty graphs;
    the wavefront kernel by default, the workgroup kernel under schedule 1."""
    gs = directed_set(700, 40, 0, 32, 0.05, 0.4)
    rng = np.random.default_rng(701)
    pairs = rng.integers(0, 40, size=(150, 2))
    check(ged, gs, pairs, costs, K, expect_words={2}, schedule=schedule,
          kinds={"kb_wave2_kernel"} if schedule == 0 else None)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("last_level", [0, 1])
def test_labelled_arcs_two_and_four_planes(ged, last_level, schedule):
    for nel, seed in ((3, 710), (12, 711)):
        gs = directed_set(seed, 30, 5, 30, 0.1, 0.3, nl=3, nel=nel)
        rng = np.random.default_rng(seed)
        check(ged, gs, rng.integers(0, 30, size=(120, 2)), NONMETRIC, 16, last_level=last_level,
              schedule=schedule)


def test_wavefront_and_workgroup_bins_together(ged):
    """One plan over directed pairs of up to 32 vertices (wavefront kernel) and larger
    ones (workgroup kernel), at K = 24, at K = 65 and 128 (two beam slots per lane) and
    at K = 129 (past the wavefront kernel's limit)."""
    gs = GraphSet.from_graphs([synth.directed_graph(715, k, 3, 32, 0.1, 0.3, 3, 3) for k in range(10)]
                              + [synth.directed_graph(716, k, 33, 60, 0.05, 0.1, 3, 3) for k in range(4)])
    pairs = [[a, b] for a in range(14) for b in range(14) if a != b][::3]
    check(ged, gs, pairs, PAPER, 24, kinds={"kb_wave2_kernel", "kb_block_kernel"})
    check(ged, gs, pairs[:30], PAPER, 65, kinds={"kb_wave2_kernel", "kb_block_kernel"})
    check(ged, gs, pairs[:30], PAPER, 128, kinds={"kb_wave2_kernel", "kb_block_kernel"})
    check(ged, gs, pairs[:30], PAPER, 129, kinds={"kb_block_kernel"})


@pytest.mark.parametrize("n_lo,n_hi,words,npairs", [(33, 64, 4, 40), (65, 128, 8, 30), (129, 200, 16, 12)])
def test_row_widths(ged, n_lo, n_hi, words, npairs):
    gs = directed_set(720 + words, 12, n_lo, n_hi, 0.02, 0.08, nl=5, nel=3)
    pairs = [[a, b] for a in range(12) for b in range(12) if a != b][:npairs]
    check(ged, gs, pairs, PAPER, 8, expect_words={words})


def test_planes_from_hbm_and_candidates_in_workspace(ged):
    """Targets of 230..256 vertices with 4 label planes: (1 + 4) planes of n2 x 16 words
    exceed the LDS staging budget, so planes are read from HBM; K = 256 from a
    20-vertex source puts the candidate matrix (256 slots x n2 + 1 children) in the
    workspace."""
    big = [synth.directed_graph(730, k, 230, 256, 0.01, 0.03, 4, 12) for k in range(3)]
    small = [synth.directed_graph(731, 0, 20, 20, 0.1, 0.1, 4, 12)]
    gs = GraphSet.from_graphs(big + small)
    check(ged, gs, [[0, 1], [2, 0], [3, 2]], NONMETRIC, 4, expect_words={16})
    check(ged, gs, [[3, 1], [3, 0]], UNIT, 256, expect_words={16})


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_of_256_thread_workgroups_and_complete(ged, schedule):
    """600 pairs (more than two per CU: 256-thread workgroups under schedule 1), both last
    levels."""
    w = synth.batch_directed_10_30(600)
    check(ged, w.graphs, w.pairs, w.costs, w.K, schedule=schedule)
    check(ged, w.graphs, w.pairs[:200], w.costs, w.K, last_level=1, schedule=schedule)


@pytest.mark.parametrize("schedule", [0, 1])
def test_perpair_path(ged, schedule):
    w = synth.batch_directed_10_30(40)
    check(ged, w.graphs, w.pairs, PAPER, 32, perpair=True, schedule=schedule)


def test_two_cycles_and_reversed_arcs(ged):
    """Hand cases: an arc against its reverse (distance 0 by swapping), a 2-cycle
    against one arc, a path against a cycle."""
    def dg(n, arcs, el=None):
        return Graph(n, np.zeros(n, np.int32), np.asarray([a for a, _ in arcs], np.int32).reshape(-1),
                     np.asarray([b for _, b in arcs], np.int32).reshape(-1),
                     None if el is None else np.asarray(el, np.int32))
    gs = GraphSet.from_graphs([dg(2, [(0, 1)]), dg(2, [(1, 0)]), dg(2, [(0, 1), (1, 0)]),
                               dg(3, [(0, 1), (1, 2)]), dg(3, [(0, 1), (1, 2), (2, 0)]), dg(0, [])])
    pairs = [[0, 1], [1, 0], [2, 0], [0, 2], [3, 4], [4, 3], [5, 2], [2, 5], [5, 5]]
    res = check(ged, gs, pairs, UNIT, 4)
    assert res.dist[0] == 0 and res.dist[4] == 1


def test_symmetric_closure_matches_undirected_doubled(ged):
    """Both arcs of every edge of undirected graphs, searched as a directed database, give
    the undirected search's result with the edge costs doubled (also on the GPU's
    undirected kernels)."""
    w = synth.batch_er_10_30(200)
    g = w.graphs
    sym = GraphSet(g.n, 2 * g.m, g.voff, 2 * g.eoff, g.vlabel,
                   np.concatenate([np.concatenate([g.eu[a:b], g.ev[a:b]]) for a, b in zip(g.eoff[:-1], g.eoff[1:])]),
                   np.concatenate([np.concatenate([g.ev[a:b], g.eu[a:b]]) for a, b in zip(g.eoff[:-1], g.eoff[1:])]),
                   None)
    c = w.costs
    c2 = (c[0], c[1], c[2], 2 * c[3], 2 * c[4], 2 * c[5])
    dd = ged.Database(sym, directed=True)
    du = ged.Database(g)
    a = ged.kbest(dd, w.pairs, c, w.K)
    b = ged.kbest(du, w.pairs, c2, w.K)
    dd.close()
    du.close()
    np.testing.assert_array_equal(a.dist, b.dist)
    np.testing.assert_array_equal(a.maps, b.maps)


def test_directed_database_refusals(ged):
    gs = GraphSet.from_graphs([synth.directed_graph(740, k, 5, 10, 0.2, 0.2, 2) for k in range(3)]
                              + [synth.directed_graph(741, 0, 257, 257, 0.01, 0.01, 2)])
    db = ged.Database(gs, directed=True)
    flags = ctypes.c_uint32()
    assert ged.load().ged_db_flags(db.handle, ctypes.byref(flags)) == ged.GED_OK
    assert flags.value == ged.DB_DIRECTED
    for make in (lambda: ged.Plan(db, [[0, 3]], 4),
                 lambda: ged.Plan(db, [[0, 1]], 4, method=ged.METHOD_BIPARTITE),
                 lambda: ged.Wide(db, 0, 1, 1024),
                 lambda: ged.Server(db, 8, UNIT, method=ged.METHOD_BIPARTITE)):
        with pytest.raises(ged.GedError) as e:
            make()
        assert e.value.status == ged.GED_EUNSUPPORTED, e.value
    srv = ged.Server(db, 8, UNIT, streams=1)
    with pytest.raises(ged.GedError) as e:
        srv.submit(gs.graph(3), 0)          # a 257-vertex directed query
    assert e.value.status == ged.GED_EUNSUPPORTED
    srv.close()
    db.close()


@pytest.mark.parametrize("K", [16, 80])
def test_server_serves_directed_queries(ged, K):
    """The server over a directed database: queries of all sizes up to 256 vertices (the
    two-word wavefront class at K <= 64, the workgroup classes otherwise), from two
    concurrent clients, each result equal to the oracle's directed search."""
    import threading
    gdb = ([synth.directed_graph(770, k, 3, 32, 0.1, 0.3, 3, 3) for k in range(20)]
           + [synth.directed_graph(771, k, 33, 120, 0.03, 0.08, 3, 3) for k in range(6)]
           + [synth.directed_graph(772, k, 129, 200, 0.01, 0.03, 3, 3) for k in range(2)])
    queries = ([synth.directed_graph(773, k, 3, 32, 0.1, 0.3, 3, 3) for k in range(40)]
               + [synth.directed_graph(774, k, 33, 100, 0.03, 0.08, 3, 3) for k in range(6)]
               + [synth.directed_graph(775, 0, 140, 140, 0.01, 0.01, 3, 3)]
               + [synth.directed_graph(777, 0, 0, 0, 0.0, 0.0, 3, 3),          # empty query
                  synth.directed_graph(778, 0, 256, 256, 0.005, 0.005, 3, 3)])  # the largest order
    rng = np.random.default_rng(776)
    # small queries against small targets (wavefront class), the rest anywhere; the
    # empty query against a small target, the largest against a 129..200-vertex one
    targets = [int(rng.integers(0, 20)) if q < 40 else int(rng.integers(0, len(gdb))) for q in range(47)]
    targets += [3, len(gdb) - 1]
    db = ged.Database(GraphSet.from_graphs(gdb), directed=True)
    srv = ged.Server(db, K, PAPER, max_batch=16, streams=2)
    results = {}
    errors = []

    def client(idx):
        try:
            tickets = [(q, srv.submit(queries[q], targets[q])) for q in idx]
            for q, t in tickets:
                results[q] = srv.wait(t, timeout_us=120_000_000)
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=client, args=(list(range(c, len(queries), 2)),)) for c in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    srv.close()
    db.close()
    assert not errors, errors
    for q in range(len(queries)):
        d, m = results[q]
        rd, rm = oracle.kbest(queries[q], gdb[targets[q]], PAPER, K, directed=True)
        assert d == rd and np.array_equal(m, rm), (q, d, rd)


def test_edit_paths_of_directed_mappings(ged):
    """Edit paths of the directed search's mappings, operation for operation against the
    oracle's expansion; each pair's costs sum to its distance."""
    import torch
    gs = directed_set(750, 24, 0, 40, 0.05, 0.3, nl=3, nel=5)
    rng = np.random.default_rng(751)
    pairs = rng.integers(0, 24, size=(80, 2)).astype(np.int64)
    db = ged.Database(gs, directed=True)
    plan = ged.Plan(db, pairs, 8)
    dist, maps, _ = plan.outputs()
    plan.run(NONMETRIC, dist, maps)
    torch.cuda.synchronize()
    ops, off, cnt = ged.edit_path(db, pairs, NONMETRIC, maps)
    d = dist[:len(pairs)].cpu().numpy()
    m = maps[:plan.map_size].cpu().numpy()
    plan.close()
    db.close()
    moff = np.concatenate([[0], np.cumsum(gs.n[pairs[:, 0]])])
    for q, (a, b) in enumerate(pairs):
        ref = oracle.edit_path(gs.graph(int(a)), gs.graph(int(b)), NONMETRIC, m[moff[q]:moff[q + 1]], directed=True)
        got = ops[off[q]:off[q] + cnt[q]]
        np.testing.assert_array_equal(got, np.asarray(ref, dtype=np.int32).reshape(-1, 6))
        assert int(got[:, 5].sum()) == d[q]


def test_full_batch_sampled(ged):
    """The 4096-pair directed batch (n 10..30, K = 64) in one plan; every 8th pair
    against the oracle."""
    w = synth.batch_directed_10_30(4096)
    db = ged.Database(w.graphs, directed=True)
    res = ged.kbest(db, w.pairs, w.costs, w.K)
    db.close()
    idx = np.arange(0, len(w.pairs), 8)
    d, m, off = oracle.kbest_pairs(w.graphs, w.pairs[idx], w.costs, w.K, directed=True)
    np.testing.assert_array_equal(res.dist[idx], d)
    n1 = w.graphs.n[w.pairs[idx, 0]]
    for k, q in enumerate(idx):
        np.testing.assert_array_equal(res.mapping(q, n1[k]), m[off[k]:off[k] + n1[k]])


def test_graph_replay_and_tune(ged, tmp_path):
    """A directed plan with a wavefront bin and a workgroup bin, tuned (choices cached), then
    captured once and replayed four times with another plan's eager run between replays;
    every replay equals the oracle."""
    import torch
    gs = GraphSet.from_graphs([synth.directed_graph(760, k, 5, 32, 0.1, 0.25, 3, 2) for k in range(30)]
                              + [synth.directed_graph(761, k, 33, 50, 0.05, 0.1, 3, 2) for k in range(6)])
    rng = np.random.default_rng(762)
    pairs = rng.integers(0, 36, size=(150, 2)).astype(np.int64)
    costs, K = PAPER, 20
    d_ref, m_ref, _ = oracle.kbest_pairs(gs, pairs, costs, K, directed=True)
    db = ged.Database(gs, directed=True)
    plan = ged.Plan(db, pairs, K)
    assert {name for name, *_ in plan.bins()} == {"kb_wave2_kernel", "kb_block_kernel"}
    dist, maps, _ = plan.outputs()
    cache = str(tmp_path / "tune.txt")
    assert plan.tune(costs, dist, maps, cache_path=cache) >= 1
    other = ged.Plan(db, pairs[::-1].copy(), 7)
    od, om, _ = other.outputs()
    s = torch.cuda.Stream()
    plan.capture(costs, dist, maps, stream=s)
    for rep in range(4):
        with torch.cuda.stream(s):
            dist.fill_(-7)
            maps.fill_(-7)
        plan.replay(stream=s)
        s.synchronize()
        np.testing.assert_array_equal(dist[:len(pairs)].cpu().numpy(), d_ref)
        np.testing.assert_array_equal(maps[:plan.map_size].cpu().numpy(), m_ref)
        other.run(costs, od, om)
        torch.cuda.synchronize()
    plan.close()
    other.close()
    db.close()


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("last_level", [0, 1])
def test_large_costs(ged, schedule, last_level):
    """Costs of 2^22 and above (the wavefront kernel's full-width cost products) with
    labelled arcs, both last levels."""
    big = (4_194_304, 5_000_011, 4_500_007, 30_011, 20_021, 35_003)
    gs = directed_set(780, 24, 2, 32, 0.05, 0.3, nl=3, nel=3)
    rng = np.random.default_rng(781)
    check(ged, gs, rng.integers(0, 24, size=(80, 2)), big, 12, last_level=last_level, schedule=schedule,
          kinds={"kb_wave2_kernel"} if schedule == 0 else None)
