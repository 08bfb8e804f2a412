"""The serving loop with the bipartite method (ged_server_config.method): results
equal the bipartite oracle's, alone and in a concurrent mix over its four size
classes; a pair past n1 + n2 = 256 is refused at submit (GPU)."""
import threading

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from paper_2605_00830_amd.synth import GraphSet

pytestmark = pytest.mark.gpu

K = 16
COSTS = synth.PAPER_COSTS


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00830_amd import ged as g
    g.load()
    return g


def mix(seed, count):
    """The serving mix's graphs, every fourth replaced by a sparse 60..130-vertex
    ER graph so that all four size classes occur."""
    out = []
    for i in range(count):
        g = synth.mix_graph(seed, i)
        if i % 4 == 0 or g.n > 130:
            g = synth.er_graph(seed, 20_000 + i, 60, 130, 0.03, 0.08, 8)
        out.append(g)
    return out


def test_bipartite_server_matches_oracle(ged):
    db_graphs = mix(51, 200)
    queries = mix(52, 160)
    rng = np.random.default_rng(7)
    targets = rng.integers(0, len(db_graphs), len(queries))
    order = np.array([queries[q].n + db_graphs[t].n for q, t in enumerate(targets)])
    keep = np.nonzero(order <= 256)[0]
    assert len(set(((order[keep] + 63) // 64).tolist())) == 4   # all four size classes
    gs = GraphSet.from_graphs(db_graphs + queries)
    pairs = np.stack([len(db_graphs) + keep, targets[keep]], 1).astype(np.int64)
    d, m, off, _ = oracle.bipartite_pairs(gs, pairs, COSTS, K)
    expect = {int(q): (int(d[k]), m[off[k]:off[k] + queries[q].n].tolist()) for k, q in enumerate(keep)}
    db = ged.Database(GraphSet.from_graphs(db_graphs))
    srv = ged.Server(db, K, COSTS, max_batch=32, streams=2, method=ged.METHOD_BIPARTITE)
    alone = {}
    for q in keep[:3]:
        t = srv.submit(queries[q], int(targets[q]))
        dd, mm = srv.wait(t, timeout_us=60_000_000)
        alone[int(q)] = (dd, mm.tolist())
    tickets = {}

    def client(part):
        for q in part:
            tickets[int(q)] = srv.submit(queries[q], int(targets[q]))

    th = [threading.Thread(target=client, args=(keep[0::2],)), threading.Thread(target=client, args=(keep[1::2],))]
    for x in th:
        x.start()
    for x in th:
        x.join()
    for q, t in tickets.items():
        dd, mm = srv.wait(t, timeout_us=120_000_000)
        assert (dd, mm.tolist()) == expect[q], q
    for q, r in alone.items():
        assert r == expect[q]
    huge = synth.er_graph(53, 0, 200, 200, 0.01, 0.01, 8)
    assert huge.n + db_graphs[0].n > 256
    with pytest.raises(ged.GedError) as e:
        srv.submit(huge, 0)
    assert e.value.status == ged.GED_EUNSUPPORTED
    st = srv.stats()
    assert st["completed"] == len(keep) + len(alone)
    srv.close()
    with pytest.raises(ged.GedError) as e:
        ged.Server(db, 300, COSTS, method=ged.METHOD_BIPARTITE)
    assert e.value.status == ged.GED_EUNSUPPORTED
    with pytest.raises(ged.GedError) as e:
        ged.Server(db, K, COSTS, method=9)
    assert e.value.status == ged.GED_EINVAL
    db.close()
