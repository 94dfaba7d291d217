"""Parity on the sparse and serving workloads at the sizes built here.

* sparse: 200,000 documents over 30,522 terms (~120 nonzeros, Zipf(1.1) ids,
  log-normal weights), 1,000 queries (~40 nonzeros), inner product, M=32;
* serving mix: 1,000,000 x 96 Gaussian mixture (4,096 centres), L2, M=32,
  FP16 traversal + FP32 rerank under Poisson arrivals with mixed k and ef.
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


def test_sparse_200k():
    g = load_graph("splade1m_n200000")
    spec = synth.WORKLOADS["splade1m"]
    say("regenerating 200k sparse docs")
    ip, ids, vals = synth.sparse_zipf(0, 200_000, spec["nnz_doc"], vocab=spec["vocab"])
    qp, qi, qv = synth.sparse_zipf(0, 1000, spec["nnz_query"], vocab=spec["vocab"], which="queries")
    ix = ann.ann_index_create(g, "ip", spec["vocab"], sp_indptr=ip, sp_ids=ids, sp_vals=vals)
    try:
        sq = (torch.from_numpy(qp).cuda(), torch.from_numpy(qi.view(np.int16)).cuda(),
              torch.from_numpy(qv).cuda())
        for ef in (100, 500):
            say("sparse ef", ef, "1,000 queries in one launch")
            r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=ef, want_stats=True)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in r.items()}
            sample = np.arange(0, 1000, 40)
            sub = (np.concatenate([[0], np.cumsum(qp[sample + 1] - qp[sample])]),
                   np.concatenate([qi[qp[i]:qp[i + 1]] for i in sample]),
                   np.concatenate([qv[qp[i]:qp[i + 1]] for i in sample]))
            ref = oracle.hnsw_search(g, oracle.sparse_store(ip, ids, vals, spec["vocab"]), 10, ef,
                                     sparse_q=sub)
            assert np.array_equal(got["ids"][sample], ref["ids"])
            assert np.array_equal(got["dists"][sample], ref["keys"])
            assert np.array_equal(got["stats"][sample, 2], ref["stats"][:, 3])
            gtp = os.path.join(ROOT, "data", "splade1m_n200000", "gt.npz")
            if os.path.exists(gtp):
                gt = np.load(gtp)["ids"]
                say("sparse recall@10 ef", ef, oracle.recall_at_k(got["ids"], gt, 10))
    finally:
        ix.close()


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
