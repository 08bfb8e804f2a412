"""The serving loop: results equal the oracle's, alone and in a concurrent mix;
admission limits, backpressure and error paths (GPU)."""
import threading

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import GraphSet

pytestmark = pytest.mark.gpu

K = 64
COSTS = synth.UNIT_COSTS


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00830_amd import ged as g
    g.load()
    return g


@pytest.fixture(scope="module")
def setting(ged):
    """A small serving mix: database of 400 mix graphs, 300 query graphs."""
    db_graphs = [synth.mix_graph(41, i) for i in range(400)]
    # keep the test quick: no graph above 160 vertices
    db_graphs = [g if g.n <= 160 else synth.er_graph(41, 10_000 + i, 100, 160, 0.05, 0.2, 8)
                 for i, g in enumerate(db_graphs)]
    queries = [synth.mix_graph(42, q) for q in range(300)]
    queries = [g if g.n <= 160 else synth.er_graph(42, 10_000 + q, 100, 160, 0.05, 0.2, 8)
               for q, g in enumerate(queries)]
    rng = np.random.default_rng(3)
    targets = rng.integers(0, len(db_graphs), len(queries))
    gs = GraphSet.from_graphs(db_graphs + queries)
    pairs = np.stack([np.arange(len(db_graphs), len(db_graphs) + len(queries)), targets], 1).astype(np.int64)
    d, m, off = oracle.kbest_pairs(gs, pairs, COSTS, K)
    expect = [(int(d[q]), m[off[q]:off[q] + queries[q].n].tolist()) for q in range(len(queries))]
    db = ged.Database(GraphSet.from_graphs(db_graphs))
    yield db, queries, targets, expect
    db.close()


def test_mix_matches_oracle_and_alone(ged, setting):
    db, queries, targets, expect = setting
    srv = ged.Server(db, K, COSTS, max_batch=64, streams=3)
    # each of a few queries alone first
    alone = {}
    for q in (0, 7, 42, 299):
        t = srv.submit(queries[q], int(targets[q]))
        d, m = srv.wait(t, timeout_us=60_000_000)
        alone[q] = (d, m.tolist())
    # then everything at once from two client threads, in the mix
    tickets = {}

    def client(lo, hi):
        for q in range(lo, hi):
            tickets[q] = srv.submit(queries[q], int(targets[q]))

    th = [threading.Thread(target=client, args=(0, 150)), threading.Thread(target=client, args=(150, 300))]
    for x in th:
        x.start()
    for x in th:
        x.join()
    got = {}
    for q, t in tickets.items():
        d, m = srv.wait(t, timeout_us=120_000_000)
        got[q] = (d, m.tolist())
    for q in range(len(queries)):
        assert got[q] == expect[q], q
    for q, r in alone.items():
        assert r == got[q] == expect[q]
    st = srv.stats()
    assert st["completed"] == st["submitted"] == 304
    assert st["batch_peak"] <= 64 and st["launches"] >= 5
    assert st["inflight"] == 0 and st["queued"] == 0
    srv.close()


def test_admission_limits_and_backpressure(ged, setting):
    db, queries, targets, expect = setting
    srv = ged.Server(db, K, COSTS, max_inflight=2, max_batch=1, streams=2, queue_capacity=3)
    tickets, busy = [], 0
    for q in range(60):
        try:
            tickets.append((q, srv.submit(queries[q], int(targets[q]))))
        except ged.GedError as e:
            assert e.status == ged.GED_EBUSY
            busy += 1
    for q, t in tickets:
        d, m = srv.wait(t, timeout_us=120_000_000)
        assert (d, m.tolist()) == expect[q]
    st = srv.stats()
    assert busy > 0 and st["rejected_busy"] == busy
    assert st["inflight_peak"] <= 2 and st["batch_peak"] == 1
    srv.close()


def test_server_errors(ged, setting):
    db, queries, targets, expect = setting
    with pytest.raises(ged.GedError) as e:
        ged.Server(db, K, COSTS, hbm_budget=1 << 20)
    assert e.value.status == ged.GED_ENOMEM
    with pytest.raises(ged.GedError) as e:
        ged.Server(db, 0, COSTS)
    assert e.value.status == ged.GED_EINVAL
    srv = ged.Server(db, K, COSTS, streams=1)
    with pytest.raises(ged.GedError) as e:
        srv.submit(queries[0], db.count)
    assert e.value.status == ged.GED_EINVAL
    bad = synth.Graph(2, np.zeros(2, np.int32), np.array([0], np.int32), np.array([1], np.int32),
                      np.array([99], np.int32))
    with pytest.raises(ged.GedError) as e:
        srv.submit(bad, 0)
    assert e.value.status == ged.GED_EINVAL and "label" in str(e.value)
    with pytest.raises(ged.GedError) as e:
        srv.poll(123456)
    assert e.value.status == ged.GED_EINVAL
    # a map buffer that is too small keeps the ticket
    big = max(range(len(queries)), key=lambda q: queries[q].n)
    t = srv.submit(queries[big], int(targets[big]))
    import ctypes
    d, n1 = ctypes.c_int32(), ctypes.c_int32()
    small = np.zeros(1, np.int32)
    st = ged.load().ged_server_wait(srv._h, ctypes.c_uint64(t), -1, ctypes.byref(d), small.ctypes.data, 1,
                                    ctypes.byref(n1), None)
    assert st == ged.GED_EINVAL
    dd, mm = srv.wait(t)
    assert (dd, mm.tolist()) == expect[big]
    srv.close()


def test_destroy_with_queued_queries(ged, setting):
    db, queries, targets, _ = setting
    srv = ged.Server(db, K, COSTS, max_inflight=1, max_batch=1, streams=1)
    for q in range(40):
        srv.submit(queries[q], int(targets[q]))
    srv.close()   # finishes the admitted query, cancels the rest, frees everything


def test_batch_submit_and_collect(ged, setting):
    db, queries, targets, expect = setting
    recs, keep = ged.pack_queries(GraphSet.from_graphs(queries))
    srv = ged.Server(db, K, COSTS, max_batch=32, streams=2)
    tickets = srv.submit_batch(recs, targets)
    assert len(tickets) == len(queries)
    pos = {int(t): q for q, t in enumerate(tickets)}
    seen = set()
    while len(seen) < len(queries):
        r = srv.collect(max_count=50, timeout_us=60_000_000, with_maps=True)
        assert r is not None
        tk, d, times, maps = r
        off = 0
        for k in range(len(tk)):
            q = pos[int(tk[k])]
            n1 = queries[q].n
            assert (int(d[k]), maps[off:off + n1].tolist()) == expect[q]
            off += n1
            assert times[k, 1] >= times[k, 0] > 0
            assert q not in seen
            seen.add(q)
    assert srv.collect(timeout_us=1000) is None
    srv.close()


def test_beam_of_128(ged):
    """K = 128: queries of up to 64 vertices take the two-slot wavefront kernel (the
    two-word class; there is no one-word class above 64 slots), larger ones the
    workgroup classes; every result equals the oracle's."""
    db_graphs = [synth.er_graph(51, i, 5, 90, 0.05, 0.25, 4) for i in range(50)]
    queries = [synth.er_graph(52, q, 5, 80, 0.05, 0.25, 4) for q in range(70)]
    targets = np.random.default_rng(53).integers(0, len(db_graphs), len(queries))
    gs = GraphSet.from_graphs(db_graphs + queries)
    pairs = np.stack([np.arange(len(db_graphs), len(db_graphs) + len(queries)), targets], 1).astype(np.int64)
    print(f"  case: server at K=128, {len(queries)} queries of 5..80 vertices", flush=True)
    d, m, off = oracle.kbest_pairs(gs, pairs, COSTS, 128)
    db = ged.Database(GraphSet.from_graphs(db_graphs))
    srv = ged.Server(db, 128, COSTS, max_batch=16, streams=2)
    tickets = [srv.submit(queries[q], int(targets[q])) for q in range(len(queries))]
    for q, t in enumerate(tickets):
        dd, mm = srv.wait(t, timeout_us=120_000_000)
        assert (dd, mm.tolist()) == (int(d[q]), m[off[q]:off[q] + queries[q].n].tolist()), q
    st = srv.stats()
    assert st["completed"] == len(queries)
    srv.close()
    db.close()
