"""The directed input generators (CPU): graphs are simple directed graphs (no
self-loop, no repeated arc, both arcs of a pair allowed), independent of
generation order, and the workloads have the stated shapes."""
import numpy as np

from paper_2605_00830_amd import synth


def test_directed_graph_is_simple_and_seeded():
    seen_two_cycle = False
    for k in range(40):
        g = synth.directed_graph(11, k, 0, 30, 0.05, 0.4, 4, 3)
        assert 0 <= g.n <= 30 and g.vlabel.shape == (g.n,)
        arcs = list(zip(g.eu.tolist(), g.ev.tolist()))
        assert all(a != b and 0 <= a < g.n and 0 <= b < g.n for a, b in arcs)
        assert len(set(arcs)) == len(arcs)
        seen_two_cycle |= any((b, a) in set(arcs) for a, b in arcs)
        assert g.elabel is not None and g.elabel.shape == (g.m,) and (g.elabel < 3).all()
        # counter-based: the same (seed, index) gives the same graph in any order
        h = synth.directed_graph(11, k, 0, 30, 0.05, 0.4, 4, 3)
        assert np.array_equal(g.eu, h.eu) and np.array_equal(g.ev, h.ev) and np.array_equal(g.elabel, h.elabel)
    assert seen_two_cycle


def test_directed_workloads():
    w = synth.batch_directed_10_30(64)
    assert len(w.pairs) == 64 and w.K == 64 and tuple(w.costs) == synth.UNIT_COSTS
    assert w.graphs.n.min() >= 10 and w.graphs.n.max() <= 30 and w.graphs.elabel is None
    s = synth.serve_mix_directed(300, 200)
    assert s.meta == {"ndb": 300, "directed": True}
    assert len(s.pairs) == 200 and (s.pairs[:, 0] == np.arange(300, 500)).all()
    assert (s.pairs[:, 1] >= 0).all() and (s.pairs[:, 1] < 300).all()
    n = np.asarray(s.graphs.n)
    assert n.min() >= 10 and n.max() <= 256
    assert ((n <= 30).mean() > 0.35) and (((n >= 33) & (n <= 70)).mean() > 0.35)
