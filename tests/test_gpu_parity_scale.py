"""Parity on the sparse and serving workloads at their configured sizes.

* sparse: 1,000,000 documents over 30,522 terms (~120 nonzeros, Zipf(1.1)
  ids, log-normal weights), 10,000 queries (~40 nonzeros) in one persistent
  launch, inner product, M=32, oracle-built graph;
* serving mix: 1,000,000 x 96 Gaussian mixture (4,096 centres), L2, M=32,
  oracle-built graph, FP16 traversal + FP32 rerank under Poisson arrivals
  with mixed k and ef; and the full 10,000,000 x 96 set, whose graph the
  device builds (the oracle's sequential-batch build of 10M nodes would take
  many hours here; the device build equals the oracle's at 1M x 96 and
  1M x 768), served, with sampled requests searched again by the oracle on
  that same graph.
Sampled queries are checked bit for bit against the oracle.  Skipped when
the oracle-built graphs are not present.
"""
import os
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[parity-scale]", *a, flush=True)


def load_graph(tag):
    p = os.path.join(ROOT, "data", tag, "graph.npz")
    if not os.path.exists(p):
        pytest.skip(f"data/{tag}/graph.npz not built")
    return oracle.Graph.load(p)


@pytest.mark.parametrize("tag,n,nq", [("splade1m", 1_000_000, 10_000)])
def test_sparse_at_size(tag, n, nq):
    g = load_graph(tag)
    spec = synth.WORKLOADS["splade1m"]
    say(f"regenerating {n:,} sparse docs and {nq:,} queries")
    ip, ids, vals = synth.sparse_zipf(0, n, spec["nnz_doc"], vocab=spec["vocab"])
    qp, qi, qv = synth.sparse_zipf(0, nq, spec["nnz_query"], vocab=spec["vocab"], which="queries")
    ix = ann.ann_index_create(g, "ip", spec["vocab"], sp_indptr=ip, sp_ids=ids, sp_vals=vals)
    try:
        sq = (torch.from_numpy(qp).cuda(), torch.from_numpy(qi.view(np.int16)).cuda(),
              torch.from_numpy(qv).cuda())
        store = oracle.sparse_store(ip, ids, vals, spec["vocab"])
        for ef in (100, 500):
            say(f"sparse ef {ef}: {nq:,} queries in one launch")
            r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=ef, want_stats=True)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in r.items()}
            assert np.all(got["status"] == 0)
            sample = np.arange(0, nq, nq // 40)
            sub = (np.concatenate([[0], np.cumsum(qp[sample + 1] - qp[sample])]),
                   np.concatenate([qi[qp[i]:qp[i + 1]] for i in sample]),
                   np.concatenate([qv[qp[i]:qp[i + 1]] for i in sample]))
            ref = oracle.hnsw_search(g, store, 10, ef, sparse_q=sub)
            say(f"  {len(sample)} sampled queries against the oracle")
            assert np.array_equal(got["ids"][sample], ref["ids"])
            assert np.array_equal(got["dists"][sample], ref["keys"])
            assert np.array_equal(got["stats"][sample, 1], ref["stats"][:, 2])
            assert np.array_equal(got["stats"][sample, 2], ref["stats"][:, 3])
            gtp = os.path.join(ROOT, "data", tag, "gt.npz")
            if os.path.exists(gtp):
                gt = np.load(gtp)["ids"]
                say("sparse recall@10 ef", ef, oracle.recall_at_k(got["ids"][:gt.shape[0]], gt, 10))
    finally:
        ix.close()


def test_serving_mix_10m_x_96_sampled_against_the_oracle():
    """The configured serving mix: 10,000,000 x 96 rows, graph built on the
    device, FP16 traversal + FP32 rerank of 40 served under Poisson arrivals
    at 20,000 requests/s with k in {10, 100} and ef in {64 .. 512}; 50
    sampled served requests equal the oracle's search of the same graph,
    bit for bit, each with its own k and ef."""
    spec = synth.WORKLOADS["gmm10m"]
    n = spec["n"]
    say(f"regenerating {n:,} x 96")
    X = synth.dense_base(spec)
    Q = synth.dense_queries(spec, nq=4000)
    u = synth.level_uniforms(0, n)
    t = time.perf_counter()
    b = ann.ann_hnsw_build(torch.from_numpy(X).to("cuda:0"), "l2", spec["M"], spec["efc"], u,
                           seq_prefix=2000, batch_frac=0.02, batch_cap=2048)
    torch.cuda.empty_cache()
    say(f"graph of {n:,} nodes built on the device in {time.perf_counter() - t:.1f} s "
        f"(max level {b.max_level})")
    X16 = X.astype(np.float16).view(np.uint16)
    ix = ann.ann_index_create(b, "l2", 96, x_f32=X, x_f16=X16)
    try:
        nreq = 2000
        t_arr, qidx, ks, efs = synth.arrivals(3, nreq, 20000.0, n_pool=Q.shape[0])
        srv = ann.Server(ix, mode="f16", rerank=40, max_inflight=4096, k_max=100, ef_max=512)
        got = {}
        try:
            t0 = time.perf_counter()
            i = 0
            while len(got) < nreq:
                assert time.perf_counter() - t0 < 120
                now = time.perf_counter() - t0
                while i < nreq and t_arr[i] <= now:
                    if not srv.submit(i, Q[qidx[i]], int(ks[i]), int(efs[i])):
                        break
                    i += 1
                for c in srv.poll():
                    got[c["tag"]] = c
                time.sleep(1e-4)
        finally:
            srv.close()
        lat = np.array([(c["t_done"] - c["t_submit"]) * 1e3 for c in got.values()])
        say(f"served {nreq} requests at 20k/s offered: p50 {np.percentile(lat, 50):.2f} ms, "
            f"p99 {np.percentile(lat, 99):.2f} ms")
    finally:
        ix.close()
    g = oracle.Graph(b.n, b.M, b.M0, b.max_level, b.entry, b.levels, b.adj0, b.upper_off,
                     b.upper_adj)
    tags = sorted(got)[::40]
    say(f"{len(tags)} sampled requests searched by the oracle on the same graph")
    st = oracle.dense_store(X16, "l2", "f16")
    ref = oracle.hnsw_search(g, st, ks[tags], efs[tags], Q=Q[qidx[tags]], rerank_f32=X, rerank=40)
    for j, tg in enumerate(tags):
        kk = int(ks[tg])
        assert got[tg]["status"] == 0
        assert np.array_equal(got[tg]["ids"], ref["ids"][j, :kk]), tg
        assert np.array_equal(got[tg]["dists"], ref["keys"][j, :kk]), tg


def test_serving_mix_1m_x_96():
    g = load_graph("gmm10m_n1000000")
    spec = synth.WORKLOADS["gmm10m"]
    say("regenerating 1M x 96")
    X = synth.dense_base(spec, n=1_000_000)
    Q = synth.dense_queries(spec, nq=2000)
    X16 = X.astype(np.float16).view(np.uint16)
    ix = ann.ann_index_create(g, "l2", 96, x_f32=X, x_f16=X16)
    try:
        n = 1500
        t_arr, qidx, ks, efs = synth.arrivals(3, n, 20000.0, n_pool=Q.shape[0])
        srv = ann.Server(ix, mode="f16", rerank=40, max_inflight=4096, k_max=100, ef_max=512)
        got = {}
        try:
            t0 = time.perf_counter()
            i = 0
            while len(got) < n:
                assert time.perf_counter() - t0 < 90
                now = time.perf_counter() - t0
                while i < n and t_arr[i] <= now:
                    if not srv.submit(i, Q[qidx[i]], int(ks[i]), int(efs[i])):
                        break
                    i += 1
                for c in srv.poll():
                    got[c["tag"]] = c
                time.sleep(1e-4)
        finally:
            srv.close()
        lat = np.array([(c["t_done"] - c["t_submit"]) * 1e3 for c in got.values()])
        say(f"served {n} requests at 20k QPS offered: p50 {np.percentile(lat, 50):.2f} ms, "
            f"p99 {np.percentile(lat, 99):.2f} ms")
        # sampled requests against the oracle, each with its own k and ef
        tags = sorted(got)[::50]
        st = oracle.dense_store(X16, "l2", "f16")
        ref = oracle.hnsw_search(g, st, ks[tags], efs[tags], Q=Q[qidx[tags]], rerank_f32=X,
                                 rerank=40)
        for j, t in enumerate(tags):
            kk = int(ks[t])
            assert np.array_equal(got[t]["ids"], ref["ids"][j, :kk])
            assert np.array_equal(got[t]["dists"], ref["keys"][j, :kk])
    finally:
        ix.close()


def test_graph_build_serving_mix_1m_x_96():
    """HNSW construction on the device of the 1,000,000 x 96 L2 set (M=32,
    efC=200, 2,000 nodes one at a time, then batches of 2% up to 2,048)
    equals the oracle's stored graph list for list."""
    g = load_graph("gmm10m_n1000000")
    spec = synth.WORKLOADS["gmm10m"]
    X = synth.dense_base(spec, n=1_000_000)
    u = synth.level_uniforms(0, X.shape[0])
    say("graph construction on the device, 1,000,000 x 96")
    t = time.perf_counter()
    b = ann.ann_hnsw_build(torch.from_numpy(X).to("cuda:0"), "l2", 32, 200, u, seq_prefix=2000,
                           batch_frac=0.02, batch_cap=2048)
    say(f"built in {time.perf_counter() - t:.1f} s")
    assert b.max_level == g.max_level and b.entry == g.entry
    assert np.array_equal(b.levels, g.levels)
    assert np.array_equal(b.upper_off, g.upper_off)
    assert np.array_equal(b.upper_adj, g.upper_adj)
    assert np.array_equal(b.adj0, g.adj0)
