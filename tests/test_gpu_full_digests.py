"""Full-size parity: the GPU's distances and mappings on every pair of the
full synthetic workloads hash to the oracle's stored digests
(tests/golden/digests.json, written by tests/golden/make_digests.py, which
calls only the oracle).  On a mismatch the stored per-pair distances name
the pairs, and the oracle is rerun on the first few of them."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2605_00830_amd import synth
from tests.golden.make_digests import DIRECTED, digest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = json.load(open(os.path.join(HERE, "golden", "digests.json")))

WORKLOADS = {
    "pair_er_8x9_k16": (synth.pair_er_8x9, None),
    "batch_er_n10-30_p0.1-0.3_4096pairs_k64": (lambda: synth.batch_er_10_30(4096), None),
    "query_molecule_n10-70_1x10000_k128": (lambda: synth.query_molecule_10_70(10000), None),
    "stress_er_n100-500_p0.05-0.5_256pairs_k256": (lambda: synth.stress_er_100_500(256), None),
    "serve_mix_db100000_q100000_k64:first2000": (lambda: synth.serve_mix(100000, 2000), 2000),
    "batch_directed_n10-30_p0.05-0.15_4096pairs_k64": (lambda: synth.batch_directed_10_30(4096), None),
}


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00830_amd import ged as g
    g.load()
    return g


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_full_workload_digest(ged, name, schedule):
    if name not in DIGESTS:
        pytest.skip(f"no stored digest for {name}")
    if schedule == 1 and name.startswith("stress"):
        pytest.skip("every stress pair takes the workgroup kernel under both schedules: one run covers it")
    ref = DIGESTS[name]
    make, limit = WORKLOADS[name]
    w = make()
    pairs = w.pairs if limit is None else w.pairs[:limit]
    assert len(pairs) == ref["pairs"] and w.K == ref["K"] and list(w.costs) == ref["costs"]
    print(f"  case: {name}, {len(pairs)} pairs, schedule {schedule}", flush=True)
    directed = name in DIRECTED
    db = ged.Database(w.graphs, directed=directed)
    res = ged.kbest(db, pairs, w.costs, w.K, schedule=schedule, with_cand=True)
    db.close()
    got = digest(res.dist, res.maps)
    if got != ref["sha256"]:
        bad = []
        if "dist" in ref:
            bad = np.nonzero(res.dist != np.asarray(ref["dist"]))[0][:5].tolist()
        detail = []
        for p in bad[:3]:
            d, m, _ = oracle.kbest_pairs(w.graphs, pairs[p:p + 1], w.costs, w.K, directed=directed)
            detail.append((p, int(res.dist[p]), int(d[0])))
        pytest.fail(f"{name}: digest {got[:16]} != {ref['sha256'][:16]}; differing pairs "
                    f"(pair, gpu, oracle): {detail or bad}")
    assert int(res.dist.astype(np.int64).sum()) == ref["dist_sum"]
    if "children_sum" in ref:
        # every child the search evaluated, summed over the workload: the
        # oracle's count of generated children
        assert int(res.cand.sum()) == ref["children_sum"]
