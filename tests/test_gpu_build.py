"""HNSW construction on the device against the oracle's build, bit for bit:
levels, every adjacency list (order included), upper-layer lists, the top
level and the entry point, for sequential and batched insertion."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-build]", *a, flush=True)


def same_graph(g, ref):
    assert (g.n, g.M, g.M0) == (ref.n, ref.M, ref.M0)
    assert g.max_level == ref.max_level and g.entry == ref.entry
    assert np.array_equal(g.levels, ref.levels)
    assert np.array_equal(g.upper_off, ref.upper_off)
    bad = np.argwhere(g.adj0 != ref.adj0)
    assert bad.size == 0, f"layer-0 lists differ first at node {bad[0][0]}"
    assert np.array_equal(g.upper_adj, ref.upper_adj)


def build_both(X, metric, M, efc, u, **kw):
    ref = oracle.hnsw_build(X, metric, M, efc, u, **kw)
    g = ann.ann_hnsw_build(torch.from_numpy(X).to("cuda:0"), metric, M, efc, u, **kw)
    return g, ref


def test_sequential_l2_gmm(gmm10k):
    X = gmm10k["X"][:3000]
    u = synth.level_uniforms(0, X.shape[0])
    say("sequential build, 3,000 x 128, L2, M=16, efC=100")
    g, ref = build_both(X, "l2", 16, 100, u)
    same_graph(g, ref)


def test_batched_ip_768(vmf_small):
    """The vmf fixture's own schedule: 1,000 nodes one at a time, then
    batches of 2% of the graph (at most 256)."""
    X = vmf_small["X"]
    u = synth.level_uniforms(0, X.shape[0])
    say("batched build, 4,096 x 768, IP, M=32, efC=100")
    g = ann.ann_hnsw_build(torch.from_numpy(X).to("cuda:0"), "ip", 32, 100, u, seq_prefix=1000,
                           batch_frac=0.02, batch_cap=256)
    same_graph(g, vmf_small["graph"])


def test_batched_l2_20k():
    """Large batches (2% of the graph, up to 2,048) after a 2,000-node prefix."""
    spec = synth.WORKLOADS["gmm10k"]
    X = synth.dense_base(spec, n=20000)
    u = synth.level_uniforms(5, X.shape[0])
    say("batched build, 20,000 x 128, L2, M=16, efC=64")
    g, ref = build_both(X, "l2", 16, 64, u, seq_prefix=2000, batch_frac=0.02, batch_cap=2048)
    same_graph(g, ref)


def test_tiny_graphs():
    rng = np.random.default_rng(2)
    for n in (1, 2, 5, 40):
        X = rng.standard_normal((n, 16)).astype(np.float32)
        u = rng.random(n)
        g, ref = build_both(X, "ip", 4, 8, u)
        same_graph(g, ref)
