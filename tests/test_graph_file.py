"""The graph file written by the oracle reads back identically through the
oracle's loader and through the benchmark's own (independent) reader."""
import numpy as np

import oracle
import synth


def test_graph_file_round_trip(tmp_path):
    X = synth.gaussian_mixture(2, 2500, 32, 8, 0.3)
    g = oracle.hnsw_build(X, "l2", 8, 32, synth.level_uniforms(2, 2500))
    p = str(tmp_path / "g.npz")
    g.save(p)
    a = oracle.Graph.load(p)
    import bench
    b = bench.read_graph(p)
    for h in (a, b):
        assert (h.n, h.M, h.M0, h.max_level, h.entry) == (g.n, g.M, g.M0, g.max_level, g.entry)
        assert np.array_equal(h.adj0, g.adj0)
        assert np.array_equal(h.levels, g.levels)
        assert np.array_equal(h.upper_off, g.upper_off)
        assert np.array_equal(h.upper_adj, g.upper_adj)
