"""Pins of the oracle's HNSW build and search.

* ef >= n on a connected layer 0 must return exact brute force;
* an independent pure-Python SEARCH-LAYER (HNSW Algorithm 2, written here from
  the published algorithm) must reproduce the oracle's results and visited
  sets on small graphs with exact integer keys;
* structural invariants of the built graph;
* a 1-D line, whose heuristic neighbours are known by hand;
* batched insertion with batches of one equals sequential insertion.
"""
import heapq

import numpy as np
import pytest

import oracle
import synth
from conftest import small_int_points


def exact_keys(X, q, metric):
    Xi = X.astype(np.int64); qi = q.astype(np.int64)
    return (-(Xi @ qi)) if metric == "ip" else ((Xi - qi) ** 2).sum(1)


def gt_topk(X, Q, metric, k):
    out = []
    for q in Q:
        kk = exact_keys(X, q, metric)
        out.append(np.lexsort((np.arange(X.shape[0]), kk))[:k])
    return np.array(out)


def reachable(g):
    seen = {g.entry}
    stack = [g.entry]
    while stack:
        v = stack.pop()
        for e in g.neighbours(v, 0):
            if e not in seen:
                seen.add(int(e)); stack.append(int(e))
    return seen


def py_search(g, key, k, ef):
    """HNSW Algorithms 5 + 2 with heaps, (key, id) order; returns (ids, visited0)."""
    def layer(eps, ef, lc):
        visited = set(e for _, e in eps)
        C = list(eps); heapq.heapify(C)
        W = [(-kk, -e) for kk, e in eps]; heapq.heapify(W)    # max-heap via negation
        while C:
            c = heapq.heappop(C)
            f = (-W[0][0], -W[0][1])
            if c > f:
                break
            for e in g.neighbours(c[1], lc):
                e = int(e)
                if e in visited:
                    continue
                visited.add(e)
                ke = (key(e), e)
                f = (-W[0][0], -W[0][1])
                if len(W) < ef or ke < f:
                    heapq.heappush(C, ke); heapq.heappush(W, (-ke[0], -ke[1]))
                    if len(W) > ef:
                        heapq.heappop(W)
        res = sorted((-a, -b) for a, b in W)
        return res, visited

    eps = [(key(g.entry), g.entry)]
    for lc in range(g.max_level, 0, -1):
        res, _ = layer(eps, 1, lc)
        eps = res[:1]
    res, vis = layer(eps, max(ef, k), 0)
    return [e for _, e in res[:k]], vis


@pytest.fixture(scope="module")
def int_graph():
    X = small_int_points(11, 400, 16, -3, 4)
    Q = small_int_points(12, 25, 16, -3, 4)
    u = synth.level_uniforms(11, 400)
    g = oracle.hnsw_build(X, "l2", 6, 20, u)
    return X, Q, g


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_ef_at_least_n_equals_bruteforce(metric):
    # n <= 2M + 1: layer 0 is connected, so a non-overflowing beam is exhaustive
    X = small_int_points(21, 33, 16)
    Q = small_int_points(22, 12, 16)
    u = synth.level_uniforms(21, 33)
    g = oracle.hnsw_build(X, metric, 16, 40, u)
    assert len(reachable(g)) == 33
    r = oracle.hnsw_search(g, oracle.dense_store(X, metric), 10, 33, Q=Q)
    assert np.array_equal(r["ids"], gt_topk(X, Q, metric, 10))


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_ef_at_least_n_equals_bruteforce_larger(metric):
    X = small_int_points(31, 300, 16)
    Q = small_int_points(32, 20, 16)
    u = synth.level_uniforms(31, 300)
    g = oracle.hnsw_build(X, metric, 8, 50, u)
    reach = reachable(g)
    r = oracle.hnsw_search(g, oracle.dense_store(X, metric), 10, 300, Q=Q, visited_cap=300)
    for i, q in enumerate(Q):
        kk = exact_keys(X, q, metric)
        ids = np.array(sorted(reach))
        want = ids[np.lexsort((ids, kk[ids]))][:10]
        assert np.array_equal(r["ids"][i], want)
        vis = r["visited"][i]
        assert set(vis[vis >= 0].tolist()) == reach


def test_matches_independent_search(int_graph):
    X, Q, g = int_graph
    st = oracle.dense_store(X, "l2")
    for ef in (1, 4, 10, 37):
        r = oracle.hnsw_search(g, st, 5, ef, Q=Q, visited_cap=400)
        for i, q in enumerate(Q):
            kk = exact_keys(X, q, "l2")
            ids, vis = py_search(g, lambda e: int(kk[e]), 5, ef)
            got = r["ids"][i]
            assert got[got >= 0].tolist() == ids
            v = r["visited"][i]
            assert set(v[v >= 0].tolist()) == vis
            assert r["stats"][i, 3] == len(vis)


def test_w_final_is_top_of_visited(int_graph):
    X, Q, g = int_graph
    r = oracle.hnsw_search(g, oracle.dense_store(X, "l2"), 5, 16, Q=Q, want_w=True, visited_cap=400)
    for i, q in enumerate(Q):
        kk = exact_keys(X, q, "l2")
        vis = r["visited"][i]; vis = vis[vis >= 0]
        top = vis[np.lexsort((vis, kk[vis]))][:16]
        w = r["w_ids"][i]
        assert np.array_equal(w[w >= 0], top)


def test_graph_invariants(gmm10k):
    g = gmm10k["graph"]
    n, M, M0 = g.n, g.M, g.M0
    assert g.levels[g.entry] == g.max_level == g.levels.max()
    deg0 = (g.adj0 >= 0).sum(1)
    assert deg0.max() <= M0 and deg0.min() >= 1
    for v in range(0, n, 7):
        row = g.neighbours(v, 0)
        assert v not in row and len(set(row.tolist())) == len(row)
        assert np.all(g.adj0[v, len(row):] == -1)
        for lc in range(1, g.levels[v] + 1):
            up = g.neighbours(v, lc)
            assert len(up) <= M and v not in up
            assert np.all(g.levels[up] >= lc)
    assert np.all((g.upper_off >= 0) == (g.levels > 0))
    # level histogram: P(level >= l) = M^-l (chi-square over levels 0, 1, >=2)
    counts = np.array([(g.levels == 0).sum(), (g.levels == 1).sum(), (g.levels >= 2).sum()])
    p = np.array([1 - 1 / M, 1 / M - 1 / M ** 2, 1 / M ** 2])
    chi2 = (((counts - n * p) ** 2) / (n * p)).sum()
    assert chi2 < 13.8  # 99.9% quantile, 2 degrees of freedom


def test_line_graph_is_a_path():
    # points 0, 1, 2, ... on a line: the heuristic keeps only the nearest
    # neighbour on each side, so layer 0 is the path graph
    n = 40
    X = np.zeros((n, 16), np.float32); X[:, 0] = np.arange(n)
    u = np.zeros(n)  # everything on layer 0
    g = oracle.hnsw_build(X, "l2", 4, 16, u)
    for v in range(n):
        want = {v - 1, v + 1} & set(range(n))
        assert set(g.neighbours(v, 0).tolist()) == want


def test_batched_build_with_unit_batches_is_sequential():
    X = synth.gaussian_mixture(5, 3000, 32, 8, 0.3)
    u = synth.level_uniforms(5, 3000)
    a = oracle.hnsw_build(X, "l2", 8, 40, u)
    b = oracle.hnsw_build(X, "l2", 8, 40, u, seq_prefix=0, batch_frac=1e-9, batch_cap=1, threads=4)
    assert np.array_equal(a.adj0, b.adj0) and np.array_equal(a.upper_adj, b.upper_adj)
    c = oracle.hnsw_build(X, "l2", 8, 40, u, seq_prefix=500, batch_frac=0.05, batch_cap=64, threads=4)
    d = oracle.hnsw_build(X, "l2", 8, 40, u, seq_prefix=500, batch_frac=0.05, batch_cap=64, threads=1)
    assert np.array_equal(c.adj0, d.adj0)   # independent of the thread count


def test_recall_on_gaussian_mixture(gmm10k):
    X, Q, g = gmm10k["X"], gmm10k["Q"], gmm10k["graph"]
    st = oracle.dense_store(X, "l2")
    gt, _ = oracle.bruteforce(st, X.shape[0], 10, Q=Q)
    r = oracle.hnsw_search(g, st, 10, 64, Q=Q)
    assert oracle.recall_at_k(r["ids"], gt, 10) >= 0.95
    assert oracle.recall_at_k(gt, gt, 10) == 1.0


def test_bruteforce_matches_numpy():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((700, 48)).astype(np.float32)
    Q = rng.standard_normal((9, 48)).astype(np.float32)
    for metric in ("l2", "ip"):
        ids, ks = oracle.bruteforce(oracle.dense_store(X, metric), 700, 7, Q=Q)
        Xd = X.astype(np.float64)
        for i, q in enumerate(Q.astype(np.float64)):
            kk = (-(Xd @ q) if metric == "ip" else ((Xd - q) ** 2).sum(1)).astype(np.float32)
            want = np.lexsort((np.arange(700), kk))[:7]
            assert np.array_equal(ids[i], want)
            assert np.array_equal(ks[i], kk[want])


def test_fewer_reachable_than_k_pads():
    X = small_int_points(41, 3, 16)
    g = oracle.hnsw_build(X, "l2", 4, 8, np.zeros(3))
    r = oracle.hnsw_search(g, oracle.dense_store(X, "l2"), 5, 8, Q=X[:1])
    assert r["ids"][0, 3:].tolist() == [-1, -1] and np.isinf(r["keys"][0, 3:]).all()


def test_rerank_reorders_by_fp32_keys(vmf_small):
    X, Q, g = vmf_small["X"], vmf_small["Q"], vmf_small["graph"]
    h = oracle.to_f16(X)
    st16 = oracle.dense_store(h, "ip", "f16")
    r = oracle.hnsw_search(g, st16, 10, 64, Q=Q, rerank_f32=X, rerank=40, want_w=True)
    st32 = oracle.dense_store(X, "ip")
    for i in range(Q.shape[0]):
        w = r["w_ids"][i][:40]
        kk = oracle.keys(st32, Q[i:i + 1], w[None].astype(np.int64), "canon")[0]
        order = np.lexsort((w, kk))[:10]
        assert np.array_equal(r["ids"][i], w[order])
        assert np.array_equal(r["keys"][i], kk[order])


def test_sparse_build_ef_at_least_n_equals_bruteforce():
    # n <= 2M + 1: layer 0 is connected, so a non-overflowing beam is exhaustive
    ip, ids, vals = synth.sparse_zipf(4, 33, 12, vocab=200)
    qp, qi, qv = synth.sparse_zipf(4, 9, 6, vocab=200, which="queries")
    g = oracle.hnsw_build_sparse(ip, ids, vals, 200, 16, 40, synth.level_uniforms(4, 33))
    assert len(reachable(g)) == 33
    st = oracle.sparse_store(ip, ids, vals, 200)
    r = oracle.hnsw_search(g, st, 8, 33, sparse_q=(qp, qi, qv), kmode="exact")
    D = np.zeros((33, 200)); Qd = np.zeros((9, 200))
    for v in range(33):
        D[v, ids[ip[v]:ip[v + 1]]] = vals[ip[v]:ip[v + 1]]
    for v in range(9):
        Qd[v, qi[qp[v]:qp[v + 1]]] = qv[qp[v]:qp[v + 1]]
    kk = (-(Qd @ D.T)).astype(np.float32)
    want = np.array([np.lexsort((np.arange(33), row))[:8] for row in kk])
    assert np.array_equal(r["ids"], want)
