"""The serving loop on the serving mix at full database size (GPU): the first 2000
queries of the mix (100,000 database graphs of 10..500 vertices), submitted as a
stream and collected in completion order, give the oracle's distances and mappings
bit for bit -- the stored digest of tests/golden/digests.json, written by
tests/golden/make_digests.py, which calls only the oracle."""
import json
import os

import numpy as np
import pytest

from paper_2605_00830_amd import synth
from tests.golden.make_digests import digest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NAME = "serve_mix_db100000_q100000_k64:first2000"


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00830_amd import ged as g
    g.load()
    return g


def test_serving_mix_matches_oracle_digest(ged):
    ref = json.load(open(os.path.join(HERE, "golden", "digests.json")))[NAME]
    nq = ref["pairs"]
    w = synth.serve_mix(100000, nq)
    assert w.K == ref["K"] and list(w.costs) == ref["costs"]
    ndb = w.meta["ndb"]
    db = ged.Database(w.graphs.slice(0, ndb))
    qgs = w.graphs.slice(ndb, ndb + nq)
    recs, keep = ged.pack_queries(qgs)
    targets = np.ascontiguousarray(w.pairs[:nq, 1])
    print(f"  case: {NAME}, {nq} queries, 2 streams per class", flush=True)
    srv = ged.Server(db, w.K, w.costs, hbm_budget=4 << 30, streams=2, max_batch=256)
    tickets = srv.submit_batch(recs, targets)
    assert len(tickets) == nq
    pos = {int(t): q for q, t in enumerate(tickets)}
    dist = np.full(nq, -7, np.int64)
    maps = [None] * nq
    seen = 0
    while seen < nq:
        r = srv.collect(max_count=1024, timeout_us=120_000_000, with_maps=True)
        assert r is not None, "no query finished within two minutes"
        tk, d, times, mp = r
        off = 0
        for k in range(len(tk)):
            q = pos[int(tk[k])]
            n1 = int(qgs.n[q])
            dist[q] = d[k]
            maps[q] = mp[off:off + n1].copy()
            off += n1
        seen += len(tk)
    srv.close()
    db.close()
    got = digest(dist.astype(np.int32), np.concatenate(maps) if maps else np.zeros(0, np.int32))
    assert int(dist.sum()) == ref["dist_sum"]
    if "dist" in ref:
        bad = np.nonzero(dist != np.asarray(ref["dist"]))[0]
        assert bad.size == 0, f"queries {bad[:10].tolist()} differ from the oracle"
    assert got == ref["sha256"]
