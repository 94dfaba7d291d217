"""Build and cache the index inputs of a workload with the CPU oracle.

Test infrastructure: everything written here comes from ``oracle`` and
``synth`` only.  The GPU library reads the cached arrays as plain inputs
(graph, storage copies, PQ codebook and codes) and never computes them.

Usage:  python -m oracle.build_index <workload> [--n N] [--threads T] [--what graph,gt,...]

Files go to ``data/<workload>[_n<N>]/`` at the repository root:
  graph.npz      HNSW graph in the exchange layout (oracle.Graph.save)
  gt.npz         exact top-100 ids/keys of the queries (EXACT keys, (key, id) order)
  pq.npz         PQ codebook f32[m,256,dsub] and codes u8[n,m]
  fp8.npz        per-row scaled E4M3 codes and scales
  ivf.npz        IVF coarse centroids f32[nlist,d] and inverted lists
                 (list_off i64[nlist+1], list_ids i32[n])
The base vectors and queries are not stored: ``synth`` regenerates them.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# IVF coarse quantizer: lists and training-sample size per workload.
IVF_NLIST = 1024
IVF_SAMPLE = 100_000

# Batched insertion keeps the searches of one batch against a frozen graph;
# the first SEQ_PREFIX nodes go in one at a time.
SEQ_PREFIX = 2000
BATCH_FRAC = 0.02
BATCH_CAP = 2048


def data_dir(workload, n=None):
    spec = synth.WORKLOADS[workload]
    tag = workload if (n is None or n == spec["n"]) else f"{workload}_n{n}"
    return os.path.join(ROOT, "data", tag)


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def build_sparse_graph(workload, n, threads):
    spec = synth.WORKLOADS[workload]
    ip, ids, vals = synth.sparse_zipf(0, n, spec["nnz_doc"], vocab=spec["vocab"])
    u = synth.level_uniforms(0, n)
    log(f"sparse graph {workload} n={n} nnz={ip[-1]} M={spec['M']} efC={spec['efc']}")
    t = time.time()
    seq = n if n <= 20000 else SEQ_PREFIX
    g = oracle.hnsw_build_sparse(ip, ids, vals, spec["vocab"], spec["M"], spec["efc"], u,
                                 seq_prefix=seq, batch_frac=BATCH_FRAC, batch_cap=BATCH_CAP,
                                 threads=threads)
    log(f"graph built in {time.time() - t:.1f}s max_level={g.max_level} entry={g.entry} "
        f"mean_deg0={(g.adj0 >= 0).sum(1).mean():.2f}")
    return g


def sparse_gt(workload, n, nq, k=100, threads=None):
    """Exact top-k of the sparse queries by a full EXACT scan (oracle)."""
    spec = synth.WORKLOADS[workload]
    ip, ids, vals = synth.sparse_zipf(0, n, spec["nnz_doc"], vocab=spec["vocab"])
    qp, qi, qv = synth.sparse_zipf(0, nq, spec["nnz_query"], vocab=spec["vocab"], which="queries")
    st = oracle.sparse_store(ip, ids, vals, spec["vocab"])
    return oracle.bruteforce(st, n, k, sparse_q=(qp, qi, qv), kmode="exact", threads=threads)


def build_graph(workload, n, threads):
    spec = synth.WORKLOADS[workload]
    X = synth.dense_base(spec, n=n)
    u = synth.level_uniforms(0, n)
    log(f"graph {workload} n={n} d={spec['d']} M={spec['M']} efC={spec['efc']}")
    t = time.time()
    seq = n if n <= 20000 else SEQ_PREFIX
    g = oracle.hnsw_build(X, spec["metric"], spec["M"], spec["efc"], u, seq_prefix=seq,
                          batch_frac=BATCH_FRAC, batch_cap=BATCH_CAP, threads=threads)
    log(f"graph built in {time.time() - t:.1f}s max_level={g.max_level} entry={g.entry} "
        f"mean_deg0={(g.adj0 >= 0).sum(1).mean():.2f}")
    return g, X


def exact_topk(X, Q, metric, k=100, pre=256, block=256):
    """Exact (key, id) top-k: FP32 GEMM preselection, FP64 rescoring.

    The FP32 preselection keeps `pre` candidates; the FP64 rescoring then
    orders them by (key, id).  The gap between the k-th EXACT key and the
    worst preselected one is checked against the FP32 GEMM error bound, and
    queries failing the check are rescored by a full FP64 scan.
    """
    n, d = X.shape
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.int64); keys = np.empty((nq, k), np.float32)
    Xd = None
    xmax = float(np.abs(X).max())
    x2max = float((X.astype(np.float64) ** 2).sum(1).max())
    for b0 in range(0, nq, block):
        q = Q[b0:b0 + block]
        if metric == "ip":
            s = -(q @ X.T)
        else:
            s = (q * q).sum(1)[:, None] - 2.0 * (q @ X.T) + (X * X).sum(1)[None, :]
        cand = np.argpartition(s, pre, axis=1)[:, :pre]
        for j in range(q.shape[0]):
            c = np.sort(cand[j])
            qd = q[j].astype(np.float64)
            xc = X[c].astype(np.float64)
            kk = -(xc @ qd) if metric == "ip" else ((xc - qd) ** 2).sum(1)
            kk32 = kk.astype(np.float32)
            order = np.lexsort((c, kk32))
            # certification: every non-candidate has FP32 score >= max over
            # candidates; with the GEMM error bound (d * 2^-23 * sum|terms|)
            # the k-th exact key must stay below that threshold.
            thr = s[j][cand[j]].max()
            if metric == "ip":
                mag = np.abs(qd).sum() * xmax
            else:
                mag = (qd * qd).sum() + x2max + 2.0 * np.abs(qd).sum() * xmax
            bound = d * 2.0 ** -21 * (mag + 1.0)
            if kk32[order[k - 1]] + bound >= thr:
                if Xd is None:
                    Xd = X.astype(np.float64)
                full = -(Xd @ qd) if metric == "ip" else ((Xd - qd) ** 2).sum(1)
                f32 = full.astype(np.float32)
                o = np.lexsort((np.arange(n), f32))[:k]
                ids[b0 + j] = o; keys[b0 + j] = f32[o]
            else:
                ids[b0 + j] = c[order[:k]]; keys[b0 + j] = kk32[order[:k]]
    return ids, keys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--what", default="graph,gt")
    ap.add_argument("--nq", type=int, default=None)
    a = ap.parse_args(argv)
    spec = synth.WORKLOADS[a.workload]
    n = a.n or spec["n"]
    out = data_dir(a.workload, a.n)
    os.makedirs(out, exist_ok=True)
    what = set(a.what.split(","))
    X = None
    if spec["kind"] == "sparse":
        if "graph" in what:
            g = build_sparse_graph(a.workload, n, a.threads)
            g.save(os.path.join(out, "graph.npz"))
            log("wrote", os.path.join(out, "graph.npz"))
        if "gt" in what:
            t = time.time()
            ids, keys = sparse_gt(a.workload, n, a.nq or spec["nq"], threads=a.threads)
            np.savez(os.path.join(out, "gt.npz"), ids=ids, keys=keys)
            log(f"gt in {time.time() - t:.1f}s")
        return
    if "graph" in what:
        g, X = build_graph(a.workload, n, a.threads)
        g.save(os.path.join(out, "graph.npz"))
        log("wrote", os.path.join(out, "graph.npz"))
    if "gt" in what:
        if X is None:
            X = synth.dense_base(spec, n=n)
        Q = synth.dense_queries(spec, nq=a.nq)
        t = time.time()
        ids, keys = exact_topk(X, Q, spec["metric"])
        np.savez(os.path.join(out, "gt.npz"), ids=ids, keys=keys)
        log(f"gt in {time.time() - t:.1f}s")
    if "pq" in what:
        if X is None:
            X = synth.dense_base(spec, n=n)
        sample, init = synth.pq_sample(0, n, 100_000, 256)
        t = time.time()
        cb, iters, obj = oracle.pq_train(X, 64, 256, sample, init, 25, threads=a.threads)
        codes = oracle.pq_encode(X, cb, threads=a.threads)
        np.savez(os.path.join(out, "pq.npz"), codebook=cb, codes=codes, objective=obj)
        log(f"pq trained ({iters} iterations) and encoded in {time.time() - t:.1f}s")
    if "fp8" in what:
        if X is None:
            X = synth.dense_base(spec, n=n)
        codes, scale = oracle.encode_fp8_rows(X, threads=a.threads)
        np.savez(os.path.join(out, "fp8.npz"), codes=codes, scale=scale)
        log("fp8 copy written")
    if "ivf" in what:
        if X is None:
            X = synth.dense_base(spec, n=n)
        nlist = min(IVF_NLIST, n)
        sample, init = synth.ivf_sample(0, n, IVF_SAMPLE, nlist)
        t = time.time()
        cent, iters, obj = oracle.ivf_train(X, nlist, sample, init, 25, threads=a.threads)
        log(f"ivf trained ({iters} iterations) in {time.time() - t:.1f}s")
        off, ids = oracle.ivf_lists(oracle.ivf_assign(X, cent, threads=a.threads), nlist)
        np.savez(os.path.join(out, "ivf.npz"), centroids=cent, list_off=off, list_ids=ids,
                 objective=obj, iters=iters)
        log(f"ivf lists written in {time.time() - t:.1f}s (sizes {np.diff(off).min()}..{np.diff(off).max()})")


if __name__ == "__main__":
    main()
