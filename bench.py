#!/usr/bin/env python3
"""Benchmark of batched HNSW search on one MI355X.

Workload (default `vmf1m`): 1,000,000 unit-norm FP32 vectors, d = 768, from a
1,024-cluster von Mises-Fisher mixture (kappa 50), inner product, HNSW with
M = 32 (M0 = 64) built by the CPU oracle on the FP32 originals; 10,000
queries from the same mixture; k = 10.  The inputs are synthetic stand-ins
for the paper's MS MARCO embedding sets (Section 3, Table 1), regenerated
from their seed; the graph and the exact ground truth come from files the
oracle wrote (oracle/build_index.py).

One step = one search of all queries in one persistent launch: FP16 rows for
the traversal, then an exact FP32 re-score of the first 4k beam entries
(the headline mode), at the smallest ef whose recall@10 reaches 0.95 in the
committed sweep (profiles/vmf1m_ef_sweep.json), or, when no ef reaches it,
the largest ef measured (the output then says recall_target_met: false).
The same search with FP32 rows (no rerank) is timed beside it.

Prints ONE JSON line with QPS, ms per step, recall@10, p50/p99 latency under
Poisson arrivals (continuous-batching server), the roofline of the search
kernel (algorithmic bytes / kernel time, HIP events on the launch stream)
and the oracle's CPU throughput on a bounded sample.  Beside the headline it
reports the exact scan on matrix cores and the IVF index over the same rows
(oracle-built lists, the smallest nprobe reaching recall@10 0.95 in
profiles/<workload>_ivf_sweep.json).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK = 157.3
FP16_MFMA_PEAK = 2500.0      # dense FP16 / BF16 matrix rate (no sparsity)
FP32_VECTOR_PEAK = 157.3
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def load_workload(name, nq=None):
    import synth
    spec = synth.WORKLOADS[name]
    ddir = os.path.join(ROOT, "data", name)
    gpath = os.path.join(ddir, "graph.npz")
    if not os.path.exists(gpath):
        raise SystemExit(f"missing {gpath}: build it with `python -m oracle.build_index {name}`")
    g = read_graph(gpath)
    t = time.time()
    X = synth.dense_base(spec)
    Q = synth.dense_queries(spec)
    if nq:
        Q = Q[:nq]
    log(f"regenerated {X.shape} base + {Q.shape} queries in {time.time() - t:.1f}s")
    gt = None
    gtp = os.path.join(ddir, "gt.npz")
    if os.path.exists(gtp):
        gt = np.load(gtp)["ids"][:Q.shape[0]]
    return spec, g, X, Q, gt


def read_graph(path):
    """The graph file: meta (n, M, M0, max_level, entry), levels u8[n], layer-0
    degrees u8[n] and ids packed in 3 little-endian bytes (lists back to back),
    upper_off i32[n], upper_adj i32[lists][M].  Returns the layout the library
    takes (layer-0 lists padded with -1 to M0)."""
    z = np.load(path)
    n, M, M0, L, e = (int(v) for v in z["meta"])

    class G:
        pass
    g = G()
    g.n, g.M, g.M0, g.max_level, g.entry = n, M, M0, L, e
    g.levels, g.upper_off, g.upper_adj = z["levels"], z["upper_off"], z["upper_adj"]
    deg = z["deg0"].astype(np.int64)
    b = z["ids0"].reshape(-1, 3).astype(np.int32)
    adj = np.full((n, M0), -1, np.int32)
    adj[np.arange(M0)[None, :] < deg[:, None]] = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16)
    g.adj0 = adj
    return g


def recall(ids, gt, k=10):
    ids = ids[:, :k]
    gt = gt[:, :k]
    hits = sum(len(set(a[a >= 0].tolist()) & set(b.tolist())) for a, b in zip(ids, gt))
    return hits / float(k * ids.shape[0])


def row_bytes(mode, d):
    return d * {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}[mode] + (4 if mode == "fp8" else 0)


def algorithmic_bytes(stats, mode, d, M0, k, rerank):
    """Bytes a search must read/write: every distance evaluation reads one row,
    every expansion one neighbour list, the rerank R FP32 rows, plus the
    query and the output rows."""
    evals = stats[:, 0].astype(np.int64)
    exps = stats[:, 1].astype(np.int64)
    w = stats[:, 3].astype(np.int64)
    rr = np.minimum(np.maximum(rerank, k), w) if rerank else np.zeros_like(w)
    per_q = evals * row_bytes(mode, d) + exps * M0 * 4 + rr * d * 4 + d * 4 + k * 12
    return int(per_q.sum())


def ivf_bytes(stats, mode, d, k, rerank, nlist):
    """Bytes an IVF search must read/write per launch: the centroids (probe
    keys), every scanned row and its id, the list offsets, the rerank rows,
    the query and the output."""
    evals = stats[:, 0].astype(np.int64)
    lists = stats[:, 1].astype(np.int64)
    rr = np.minimum(max(rerank, k), evals) if rerank else np.zeros_like(evals)
    per_q = (nlist * d * 4 + evals * (row_bytes(mode, d) + 4) + lists * 16 + rr * d * 4
             + d * 4 + k * 12)
    return int(per_q.sum())


def load_ivf(name):
    p = os.path.join(ROOT, "data", name, "ivf.npz")
    return np.load(p) if os.path.exists(p) else None


def pick_nprobe(sweep, mode_key, target=0.95):
    if not sweep or mode_key not in sweep:
        return None, None
    pts = sorted(sweep[mode_key], key=lambda r: r["nprobe"])
    for r in pts:
        if r["recall"] >= target:
            return r["nprobe"], r["recall"]
    return pts[-1]["nprobe"], pts[-1]["recall"]


class IvfTimed:
    """One IVF search configuration: K steps bracketed by events on the stream."""

    def __init__(self, ann, torch, ivf, mode, Q, k, nprobe, rerank, stream):
        self.ann, self.torch, self.ivf = ann, torch, ivf
        self.mode, self.Q, self.k, self.nprobe, self.rerank = mode, Q, k, nprobe, rerank
        self.stream = stream
        self.out = None

    def step(self):
        self.out = self.ann.ann_ivf_search(self.ivf, self.Q, self.k, self.nprobe, mode=self.mode,
                                           rerank=self.rerank, want_stats=True,
                                           stream=self.stream, out=self.out)
        return self.out



def sweep_ef(name):
    p = os.path.join(PROFILES, f"{name}_ef_sweep.json")
    if os.path.exists(p):
        return json.load(open(p))
    return None


def pick_ef(sweep, mode_key, target=0.95, default=256):
    if not sweep or mode_key not in sweep:
        return default, None
    pts = sorted(sweep[mode_key], key=lambda r: r["ef"])
    for r in pts:
        if r["recall"] >= target:
            return r["ef"], r["recall"]
    return pts[-1]["ef"], pts[-1]["recall"]


class Timed:
    """Runs one search configuration: K steps bracketed by events on the stream."""

    def __init__(self, ann, torch, ix, mode, Q, k, ef, rerank, stream):
        self.ann, self.torch, self.ix = ann, torch, ix
        self.mode, self.Q, self.k, self.ef, self.rerank, self.stream = mode, Q, k, ef, rerank, stream
        self.out = None

    def step(self, stats=False):
        r = self.ann.ann_search_ex(self.ix, self.mode, queries=self.Q, k=self.k, ef=self.ef,
                                   rerank=self.rerank, stream=self.stream, want_stats=stats,
                                   out=None if stats else self.out)
        if not stats and self.out is None:
            self.out = r
        return r

    def run(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        e1.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / steps, wall


IvfTimed.run = Timed.run


def ivf_row(ann, torch, ivf, mode, Qd, k, nprobe, rerank, stream, gt, d, nlist, steps, warmup,
            traffic=None):
    """One IVF configuration.  With one query per workgroup every scanned row
    is read from device memory for its query, so the algorithmic bytes are
    real HBM bytes and the roofline is the HBM's.  With the shared scan a
    workgroup reads each probed list once for its 8 queries: the
    per-query-equivalent bytes then exceed what crosses the HBM interface
    (the counters measure that), and the bound is the FP32 vector arithmetic
    of the scoring (2 d flops per scanned row and query)."""
    tm = IvfTimed(ann, torch, ivf, mode, Qd, k, nprobe, rerank, stream)
    ms, _ = tm.run(steps, warmup)
    nq = Qd.shape[0]
    rec = recall(tm.out["ids"].cpu().numpy(), gt, k) if gt is not None else None
    nb = ivf_bytes(tm.out["stats"].cpu().numpy(), mode, d, k, rerank, nlist)
    gbs = nb / (ms / 1e3) / 1e9
    evals = float(tm.out["stats"][:, 0].double().sum().item())
    tflops = 2.0 * evals * d / (ms / 1e3) / 1e12
    shared = mode != "pq" and 4 * min(nprobe, nlist) > nlist
    row = {"nprobe": nprobe, "qps": round(nq / (ms / 1e3), 1), "recall@10": rec,
           "ms_per_step": round(ms, 3),
           "scan": "8 queries per workgroup share LDS tiles" if shared else "one query per workgroup",
           "tflops": round(tflops, 2)}
    if shared:
        row["per_query_equivalent_GBps"] = round(gbs, 1)
        row["roofline"] = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_VECTOR_PEAK,
                           "unit": "TFLOP/s", "frac": round(tflops / FP32_VECTOR_PEAK, 4)}
    else:
        row["algorithmic_GBps"] = round(gbs, 1)
        row["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if traffic is not None:
        row["roofline"]["traffic"] = traffic
        row["hbm_traffic_GBps"] = round(traffic / (ms / 1e3) / 1e9, 1)
    return row


def serve_latency(ann, ix, Q, k, ef, mode, rerank, qps_peak, seconds=3.0, seed=0, waves=0):
    """Open-loop Poisson arrivals at half the measured peak through the
    server (per-slot admission), each of the first queries once; returns
    p50/p99 of completion - submission (host clock, ms), the offered rate, and
    p50/p99 of the device service time (claim to completion on the kernel's
    own clock).  waves > 0 sets the waves per query of the server's kernel
    (0: the index's current launch shape)."""
    import synth
    saved = ann.ann_get_launch(ix, mode)
    if waves:
        ann.ann_set_launch(ix, mode, waves_per_query=waves, slots=0,
                           lanes_per_row=saved["lanes_per_row"])
    rate = max(100.0, 0.5 * qps_peak)
    n_req = int(min(Q.shape[0] * 4, max(200, rate * seconds)))
    t_arr, qidx, _, _ = synth.arrivals(seed, n_req, rate, k_choices=(k,), ef_choices=(ef,),
                                       n_pool=Q.shape[0])
    srv = ann.Server(ix, mode=mode, rerank=rerank, max_inflight=8192, k_max=max(k, 10), ef_max=ef)
    lat, svc = [], []
    try:
        info = srv.info()
        t0 = time.perf_counter()
        i = 0
        done = 0
        while done < n_req:
            now = time.perf_counter() - t0
            while i < n_req and t_arr[i] <= now:
                if not srv.submit(i, Q[qidx[i]], k, ef):
                    break
                i += 1
            for c in srv.poll():
                lat.append((c["t_done"] - c["t_submit"]) * 1e3)
                svc.append((c["d_done"] - c["d_start"]) * 1e3)
                done += 1
            if i < n_req and t_arr[i] > now:
                time.sleep(min(2e-4, t_arr[i] - now))
    finally:
        srv.close()
        ann.ann_set_launch(ix, mode, **{k_: v for k_, v in saved.items()})
    lat, svc = np.array(lat), np.array(svc)
    return {"offered_qps": round(rate, 1), "requests": n_req,
            "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "service_p50_ms": round(float(np.percentile(svc, 50)), 2),
            "service_p99_ms": round(float(np.percentile(svc, 99)), 2),
            "slots": info["slots"], "waves_per_query": info["waves_per_query"]}


def serve_mix(ann, torch, n=None, seconds=3.0, rates=(5000, 10000, 20000, 35000, 50000),
              rerank=40):
    """The serving mix: dense vectors of 96 dimensions from a 4,096-centre
    Gaussian mixture (10,000,000 by default), HNSW M = 32, efC = 200 built on
    the device, FP16 rows + FP32 rerank; open-loop Poisson arrivals at each
    rate, every request with k in {10, 100} and ef in {64, 128, 256, 512}
    drawn uniformly.  Reports p50/p99 latency and the completion rate per
    offered rate, and checks that served results equal a direct batch search
    of the same requests."""
    import synth
    spec = synth.WORKLOADS["gmm10m"]
    n = n or spec["n"]
    t = time.perf_counter()
    X = synth.dense_base(spec, n=n)
    Q = synth.dense_queries(spec)
    log(f"serving mix: regenerated {X.shape} + {Q.shape} in {time.perf_counter() - t:.1f}s")
    Xd = torch.from_numpy(X).to("cuda:0")
    u = synth.level_uniforms(0, n)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = ann.ann_hnsw_build(Xd, spec["metric"], spec["M"], spec["efc"], u, seq_prefix=2000,
                           batch_frac=0.02, batch_cap=2048)
    build_s = time.perf_counter() - t
    del Xd
    torch.cuda.empty_cache()
    log(f"serving mix: graph built on the device in {build_s:.1f}s (max level {g.max_level})")
    ix = ann.ann_index_create(g, spec["metric"], X.shape[1], x_f32=X,
                              x_f16=X.astype(np.float16).view(np.uint16))
    out = {"n": int(n), "d": int(X.shape[1]), "M": spec["M"], "efc": spec["efc"],
           "build_seconds": round(build_s, 2), "rerank": rerank, "rates": []}
    for i_rate, rate in enumerate(rates):
        n_req = int(rate * seconds)
        t_arr, qidx, ks, efs = synth.arrivals(i_rate, n_req, rate, k_choices=(10, 100),
                                              ef_choices=(64, 128, 256, 512), n_pool=Q.shape[0])
        srv = ann.Server(ix, mode="f16", rerank=rerank, max_inflight=16384, k_max=100, ef_max=512)
        lat = np.zeros(n_req)
        svc = np.zeros(n_req)
        got = {}
        try:
            t0 = time.perf_counter()
            i = done = 0
            while done < n_req:
                now = time.perf_counter() - t0
                while i < n_req and t_arr[i] <= now:
                    if not srv.submit(i, Q[qidx[i]], int(ks[i]), int(efs[i])):
                        break
                    i += 1
                for c in srv.poll():
                    lat[c["tag"]] = (c["t_done"] - c["t_submit"]) * 1e3
                    svc[c["tag"]] = (c["d_done"] - c["d_start"]) * 1e3
                    if c["tag"] < 512:
                        got[c["tag"]] = c["ids"]
                    done += 1
                if i < n_req and t_arr[i] > now:
                    time.sleep(min(2e-4, t_arr[i] - now))
            wall = time.perf_counter() - t0
        finally:
            srv.close()
        # the first 512 requests again, as one direct batch with per-query k and ef
        m = min(512, n_req)
        r = ann.ann_search_ex(ix, "f16", queries=torch.from_numpy(Q[qidx[:m]]).to("cuda:0"),
                              k=torch.from_numpy(ks[:m]).to("cuda:0"),
                              ef=torch.from_numpy(efs[:m]).to("cuda:0"), rerank=rerank,
                              k_max=100, ef_max=512)
        direct = r["ids"].cpu().numpy()
        same = sum(bool(np.array_equal(got[j], direct[j, :ks[j]])) for j in range(m))
        # recall@10 of those requests against the exact scan on matrix cores
        gt, _, _ = ann.ann_bruteforce(ix, torch.from_numpy(Q[qidx[:m]]).to("cuda:0"), 10)
        rec = recall(direct[:, :10], gt.cpu().numpy(), 10)
        row = {"offered_qps": rate, "requests": n_req, "completed_qps": round(n_req / wall, 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "service_p50_ms": round(float(np.percentile(svc, 50)), 3),
               "service_p99_ms": round(float(np.percentile(svc, 99)), 3),
               "served_equal_direct": f"{same}/{m}", "recall@10_first_512": round(rec, 4)}
        out["rates"].append(row)
        log(f"serving mix at {rate} QPS offered: {row['completed_qps']:.0f} QPS completed, "
            f"p50 {row['p50_ms']:.2f} ms, p99 {row['p99_ms']:.2f} ms (service p50 "
            f"{row['service_p50_ms']:.2f}, p99 {row['service_p99_ms']:.2f}), same as direct {same}/{m}, "
            f"recall@10 {rec:.4f}")
    ix.close()
    return out


def sparse_sweep(ann, torch, efs=(100, 200, 300, 400, 500), nq=10000):
    """The sparse workload: the 1M-document SPLADE-shaped set (30,522 terms,
    ~120 nonzeros per document, ~40 per query, Zipf(1.1) term ids,
    log-normal weights; its first 200,000 documents when only that graph was
    built), inner product, the oracle-built graph (M = 32, efC = 200); all
    queries in one persistent launch per ef."""
    import synth
    spec = synth.WORKLOADS["splade1m"]
    ddir = os.path.join(ROOT, "data", "splade1m")
    if not os.path.exists(os.path.join(ddir, "graph.npz")):
        ddir = os.path.join(ROOT, "data", "splade1m_n200000")
    g = read_graph(os.path.join(ddir, "graph.npz"))
    n = g.n
    ip, ids, vals = synth.sparse_zipf(0, n, spec["nnz_doc"], vocab=spec["vocab"])
    qp, qi, qv = synth.sparse_zipf(0, nq, spec["nnz_query"], vocab=spec["vocab"], which="queries")
    # the ground truth file holds the exact top-100 of a draw of its own
    # query count (the generator draws whole arrays, so a smaller draw is not
    # a prefix of this one)
    gtp = os.path.join(ddir, "gt.npz")
    gt = np.load(gtp)["ids"] if os.path.exists(gtp) else None
    rq = None
    if gt is not None:
        rp, ri, rv = synth.sparse_zipf(0, gt.shape[0], spec["nnz_query"], vocab=spec["vocab"],
                                       which="queries")
        rq = (torch.from_numpy(rp).to("cuda:0"), torch.from_numpy(ri.view(np.int16)).to("cuda:0"),
              torch.from_numpy(rv).to("cuda:0"))
    ix = ann.ann_index_create(g, "ip", spec["vocab"], sp_indptr=ip, sp_ids=ids, sp_vals=vals)
    sq = (torch.from_numpy(qp).to("cuda:0"), torch.from_numpy(qi.view(np.int16)).to("cuda:0"),
          torch.from_numpy(qv).to("cuda:0"))
    nnz = np.diff(ip)
    stream = torch.cuda.Stream()
    out = {"docs": int(n), "queries": int(nq), "mean_nnz_doc": round(float(nnz.mean()), 1),
           "mean_nnz_query": round(float(np.diff(qp).mean()), 1), "rows": []}
    for ef in efs:
        r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=ef, want_stats=True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=ef, stream=stream, out=r)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        st = r["stats"].cpu().numpy()
        rec = None
        if rq is not None:
            rr = ann.ann_search_ex(ix, "sparse", sparse=rq, k=10, ef=ef)
            rec = round(recall(rr["ids"].cpu().numpy(), gt, 10), 4)
        # bytes a search must read: per evaluated document its indptr pair and
        # its nonzeros (u16 id + f32 weight), per expansion a neighbour list
        evals = st[:, 0].astype(np.int64).sum()
        exps = st[:, 1].astype(np.int64).sum()
        doc_bytes = 16 + 6 * float(nnz.mean())
        nb = evals * doc_bytes + exps * g.M0 * 4 + nq * (6 * float(np.diff(qp).mean()) + 8 + 120)
        gbs = nb / (ms / 1e3) / 1e9
        row = {"ef": ef, "qps": round(nq / (ms / 1e3), 1),
               "recall@10": rec, "recall_queries": None if gt is None else int(gt.shape[0]),
               "ms_per_step": round(ms, 3), "algorithmic_GBps": round(gbs, 1),
               "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        out["rows"].append(row)
        log(f"sparse ef={ef}: {row['qps']:.0f} QPS, recall@10 {rec}, {gbs:.0f} GB/s algorithmic")
    ix.close()
    return out


def quant_sweep(ann, torch, spec, g, X, Q, gt, efs=(100, 200, 400, 1024, 4096), rerank=100):
    """The quantized representations on the 1M x 768 set, FP32 rerank of the
    first 100, all queries in one launch per ef: PQ with 64 subspaces x 256
    centroids (the stored codebook and codes; ADC with per-query tables in
    LDS), and FP8-E4M3 rows with per-row scales (encoded on the device)."""
    z = np.load(os.path.join(ROOT, "data", "vmf1m", "pq.npz"))
    cb, codes = z["codebook"], z["codes"]
    ix = ann.ann_index_create(g, spec["metric"], X.shape[1], x_f32=X, pq_codebook=cb, pq_codes=codes)
    Qd = torch.from_numpy(Q).to("cuda:0")
    stream = torch.cuda.Stream()
    out = {"pq": {"pq_m": int(cb.shape[0]), "ksub": int(cb.shape[1]), "rerank": rerank, "rows": []},
           "fp8": {"rerank": rerank, "rows": []}}
    Xd = torch.from_numpy(X).to("cuda:0")
    f8, s8 = ann.ann_encode_fp8(Xd)
    torch.cuda.synchronize()
    del Xd
    ix8 = ann.ann_index_create(g, spec["metric"], X.shape[1], x_f32=X, x_fp8=f8.cpu().numpy(),
                               fp8_scale=s8.cpu().numpy())
    del f8, s8
    for mode, index in (("pq", ix), ("fp8", ix8)):
        out[mode]["rows"] = quant_rows(ann, torch, index, mode, Qd, gt, g, X, efs, rerank, stream,
                                       cb.shape[0])
    ix.close()
    ix8.close()
    return out


def quant_rows(ann, torch, ix, mode, Qd, gt, g, X, efs, rerank, stream, pq_m):
    rows = []
    for ef in efs:
        # the launch shape tuned for this ef on a sample of 2,048 queries
        ann.ann_set_launch(ix, mode)
        best = ann.ann_autotune(ix, mode, queries=Qd[:2048], k=10, ef=ef, rerank=rerank)
        tm = Timed(ann, torch, ix, mode, Qd, 10, ef, rerank, stream)
        ms, _ = tm.run(2, 1)
        rec = recall(tm.out["ids"].cpu().numpy(), gt, 10) if gt is not None else None
        st = tm.step(stats=True)
        torch.cuda.synchronize()
        stats = st["stats"].cpu().numpy()
        evals = stats[:, 0].astype(np.int64)
        exps = stats[:, 1].astype(np.int64)
        w = stats[:, 3].astype(np.int64)
        rr = np.minimum(max(rerank, 10), w)
        per_eval = pq_m if mode == "pq" else row_bytes("fp8", X.shape[1])
        nb = int((evals * per_eval + exps * g.M0 * 4 + rr * X.shape[1] * 4 + X.shape[1] * 4 + 120).sum())
        gbs = nb / (ms / 1e3) / 1e9
        row = {"ef": ef, "qps": round(Qd.shape[0] / (ms / 1e3), 1), "recall@10": rec,
               "ms_per_step": round(ms, 3), "algorithmic_GBps": round(gbs, 1), "launch": best}
        rows.append(row)
        log(f"{mode}+rerank{rerank} ef={ef}: {row['qps']:.0f} QPS, recall@10 {rec}, {gbs:.0f} GB/s algorithmic")
    return rows


def bruteforce_row(ann, torch, ix, Qd, k, stream, gt, n, d):
    """One exact k-NN call over all queries, timed with events on its stream."""
    try:
        ann.ann_bruteforce(ix, Qd[:256], k)          # warm the row norms and scratch
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        bids, _, cert = ann.ann_bruteforce(ix, Qd, k, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
    except ann.AnnError as e:
        log(f"bruteforce skipped: {e}")
        return None
    bms = e0.elapsed_time(e1)
    flops = 2.0 * Qd.shape[0] * n * d
    c = cert.cpu().numpy()
    # the scan's contraction runs on FP16 matrix cores when that pass
    # certifies the queries (flag 2), on FP32 ones for the rest (flag 1)
    half = float((c == 2).mean())
    peak = FP16_MFMA_PEAK if half > 0.5 else FP32_MFMA_PEAK
    bf = {"ms": round(bms, 2), "tflops": round(flops / (bms / 1e3) / 1e12, 1),
          "peak_tflops": peak, "peak_dtype": "f16" if half > 0.5 else "f32",
          "frac": round(flops / (bms / 1e3) / 1e12 / peak, 4),
          "certified": float((c != 0).mean()), "certified_by_fp16_pass": half,
          "recall@10_vs_oracle_gt": recall(bids.cpu().numpy(), gt, k) if gt is not None else None}
    log(f"bruteforce: {bms:.1f} ms, {bf['tflops']} TFLOP/s, certified {bf['certified']:.4f}, "
        f"agreement with oracle GT {bf['recall@10_vs_oracle_gt']}")
    return bf


def host_threads():
    """Threads the host gives this process (OMP_NUM_THREADS when set, else the CPUs it may use)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def cpu_baseline(g, X, Q, mode, ef, k, rerank, budget_s=20.0, single_s=10.0, exact_s=8.0):
    """The oracle's search (same mode, ef, rerank) on a sample of queries, on
    all host threads (OpenMP across queries), and on one thread (the paper's
    setting) for a shorter sample; then the same search with EXACT keys (FP64
    sums rounded once) on all host threads, the oracle's reference mode."""
    import oracle
    g = oracle.Graph(g.n, g.M, g.M0, g.max_level, g.entry, g.levels, g.adj0, g.upper_off,
                     g.upper_adj)
    threads = host_threads()
    if mode == "f16":
        st = oracle.dense_store(X.astype(np.float16).view(np.uint16), "ip", "f16")
    else:
        st = oracle.dense_store(X, "ip")
    probe = min(threads, Q.shape[0])
    t = time.perf_counter()
    oracle.hnsw_search(g, st, k, ef, Q=Q[:probe], rerank_f32=X if rerank else None, rerank=rerank,
                       threads=threads)
    dt = time.perf_counter() - t
    per = dt / probe
    m = int(max(probe, min(Q.shape[0], budget_s / max(per, 1e-6))))
    t = time.perf_counter()
    oracle.hnsw_search(g, st, k, ef, Q=Q[:m], rerank_f32=X if rerank else None, rerank=rerank,
                       threads=threads)
    dt = time.perf_counter() - t
    out = {"value": m / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"first {m} of {Q.shape[0]} queries, same graph, mode, ef and rerank, "
                     f"{dt:.1f}s"}
    # one thread: as many of the first queries as fit the shorter budget (at least one)
    n1, t = 0, time.perf_counter()
    while n1 < Q.shape[0] and (n1 == 0 or time.perf_counter() - t < single_s):
        oracle.hnsw_search(g, st, k, ef, Q=Q[n1:n1 + 1], rerank_f32=X if rerank else None,
                           rerank=rerank, threads=1)
        n1 += 1
    dt1 = time.perf_counter() - t
    single = {"value": n1 / dt1, "unit": "queries/s", "threads": 1,
              "sample": f"first {n1} queries, {dt1:.1f}s"}
    # EXACT keys: whole rounds of one query per thread until the budget is spent
    ne, t = 0, time.perf_counter()
    while ne < Q.shape[0] and (ne == 0 or time.perf_counter() - t < exact_s):
        b = min(probe, Q.shape[0] - ne)
        oracle.hnsw_search(g, st, k, ef, Q=Q[ne:ne + b], kmode="exact",
                           rerank_f32=X if rerank else None, rerank=rerank,
                           rerank_kmode="exact", threads=threads)
        ne += b
    dte = time.perf_counter() - t
    exact = {"value": ne / dte, "unit": "queries/s", "threads": threads,
             "sample": f"first {ne} queries, EXACT keys and rerank, {dte:.1f}s"}
    return out, single, exact


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="vmf1m")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--ef", type=int, default=None, help="ef of the headline mode")
    ap.add_argument("--ef-f32", type=int, default=None)
    ap.add_argument("--mode", default="f16")
    ap.add_argument("--rerank", type=int, default=40)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of tuning them on a sample")
    ap.add_argument("--tune-nq", type=int, default=3072,
                    help="queries of the sample the autotuner times each shape on")
    ap.add_argument("--launch", default=None, metavar="SLOTS,LANES,WAVES[,BUFFER]",
                    help="fixed launch shape of the headline mode instead of the autotuner's "
                         "(for profiler runs: the same shape the bench line reports)")
    ap.add_argument("--serve-waves", type=int, default=4,
                    help="waves per query of the serving kernel (0: the tuned shape); at half "
                         "load fewer requests are in flight, and 4 waves each gave the lowest "
                         "latency (measured: p99 188 ms vs 243 ms with 2)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline mode (for profiler runs)")
    ap.add_argument("--build", action="store_true",
                    help="build the workload's HNSW graph on the device, time it and compare it "
                         "with the stored graph; prints one JSON line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="copy BYTES between two device buffers 3 times and exit (the plain "
                         "copy that scales the HBM traffic counters)")
    ap.add_argument("--ivf-sweep", default=None, help="comma-separated nprobe values: write the "
                    "IVF sweep file (profiles/<workload>_ivf_sweep.json)")
    ap.add_argument("--ivf-only", action="store_true",
                    help="time only the IVF search at its chosen nprobe (for profiling)")
    ap.add_argument("--no-ivf", action="store_true")
    ap.add_argument("--bf-only", action="store_true",
                    help="time only the exact k-NN scan over all queries (for profiling)")
    ap.add_argument("--serve-mix", action="store_true",
                    help="only the serving mix: 10M x 96 graph built on the device, Poisson "
                    "arrivals at 5k-50k QPS with mixed k and ef; prints one JSON line")
    ap.add_argument("--serve-mix-n", type=int, default=None)
    ap.add_argument("--quant", action="store_true",
                    help="only PQ-ADC and FP8 rows + FP32 rerank of 100 on the 1M x 768 set")
    ap.add_argument("--sparse", action="store_true",
                    help="only the sparse workload (1M SPLADE-shaped documents), ef 100-500")
    ap.add_argument("--sweep", default=None, help="comma-separated ef values: write the sweep file")
    ap.add_argument("--sweep-out", default=None, help="where the sweep JSON goes "
                    "(default profiles/<workload>_ef_sweep.json)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (every index here "
              "fits one MI355X: queries would be split across replicas)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2501_06121_amd as ann
    assert torch.cuda.is_available(), "needs a GPU"
    if a.copy_calibration:
        src = torch.ones(a.copy_calibration, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.copy_calibration, "copies": 3}), flush=True)
        return
    if a.serve_mix:
        print(json.dumps({"serve_mix": serve_mix(ann, torch, n=a.serve_mix_n)}), flush=True)
        return
    if a.sparse:
        print(json.dumps({"sparse": sparse_sweep(ann, torch)}), flush=True)
        return
    spec, g, X, Q, gt = load_workload(a.workload, a.nq)
    if a.quant:
        print(json.dumps(quant_sweep(ann, torch, spec, g, X, Q, gt)), flush=True)
        return
    if a.build:
        build_bench(ann, torch, spec, g, X)
        return
    d, k = X.shape[1], a.k
    t = time.time()
    x16 = X.astype(np.float16).view(np.uint16)
    ix = ann.ann_index_create(g, spec["metric"], d, x_f32=X, x_f16=x16)
    log(f"index on device in {time.time() - t:.1f}s ({ix.info()['device_bytes'] / 2**30:.2f} GiB)")
    dev = "cuda:0"
    Qd = torch.from_numpy(Q).to(dev)
    stream = torch.cuda.Stream()
    if a.bf_only:
        print(json.dumps({"bruteforce_mfma": bruteforce_row(ann, torch, ix, Qd, k, stream, gt,
                                                            X.shape[0], d)}), flush=True)
        return

    ivf_data = load_ivf(a.workload)
    ivf = None
    if ivf_data is not None and not a.no_ivf:
        ivf = ann.ann_ivf_create(ix, ivf_data["centroids"], ivf_data["list_off"], ivf_data["list_ids"])
        nlist = int(ivf_data["centroids"].shape[0])
    if a.ivf_sweep:
        res = {}
        for key, mode, rr in (("f16+rerank", "f16", a.rerank), ("f32", "f32", 0)):
            pts = []
            for npb in (int(v) for v in a.ivf_sweep.split(",")):
                row = ivf_row(ann, torch, ivf, mode, Qd, k, npb, rr, stream, gt, d, nlist, 1, 1)
                pts.append({"nprobe": npb, "recall": row["recall@10"], "qps": row["qps"],
                            "scan": row["scan"], "roofline": row["roofline"]})
                log(f"ivf sweep {key} nprobe={npb} recall@10={row['recall@10']:.4f} "
                    f"qps={row['qps']:.0f} {row['roofline']}")
            res[key] = pts
        path = os.path.join(PROFILES, f"{a.workload}_ivf_sweep.json")
        with open(path, "w") as f:
            json.dump({"workload": a.workload, "k": k, "rerank": a.rerank, "nlist": nlist, **res}, f,
                      indent=1)
        return
    ivf_sweep = None
    p_sw = os.path.join(PROFILES, f"{a.workload}_ivf_sweep.json")
    if os.path.exists(p_sw):
        ivf_sweep = json.load(open(p_sw))
    if a.ivf_only:
        npb, _ = pick_nprobe(ivf_sweep, "f16+rerank")
        row = ivf_row(ann, torch, ivf, a.mode, Qd, k, npb or 64, a.rerank, stream, gt, d, nlist,
                      a.steps, a.warmup)
        print(json.dumps({"ivf": row, "mode": a.mode, "rerank": a.rerank}), flush=True)
        return

    if a.sweep:
        res = {}
        for key, mode, rr in (("f16+rerank", "f16", a.rerank), ("f32", "f32", 0)):
            pts = []
            for ef in (int(v) for v in a.sweep.split(",")):
                tm = Timed(ann, torch, ix, mode, Qd, k, ef, rr, stream)
                ms, _ = tm.run(1, 1)
                r = recall(tm.out["ids"].cpu().numpy(), gt, k)
                pts.append({"ef": ef, "recall": r, "qps": Q.shape[0] / (ms / 1e3)})
                log(f"sweep {key} ef={ef} recall@10={r:.4f} qps={pts[-1]['qps']:.0f}")
            res[key] = pts
        path = a.sweep_out or os.path.join(PROFILES, f"{a.workload}_ef_sweep.json")
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump({"workload": a.workload, "k": k, "rerank": a.rerank, **res}, f, indent=1)
        return

    sweep = sweep_ef(a.workload)
    ef, _ = pick_ef(sweep, "f16+rerank") if a.ef is None else (a.ef, None)
    ef32, _ = pick_ef(sweep, "f32") if a.ef_f32 is None else (a.ef_f32, None)
    log(f"ef: {a.mode}+rerank {ef}, f32 {ef32} (smallest ef reaching recall@10 0.95 in the sweep, "
        "else the largest ef measured)")

    # launch shapes: tuned on a sample of the queries (results do not depend
    # on the shape, only the speed does)
    launch = launch32 = None
    if a.launch:
        vals = [int(v) for v in a.launch.split(",")]
        sl, ln, wv = vals[:3]
        ann.ann_set_launch(ix, a.mode, slots=sl, lanes_per_row=ln, waves_per_query=wv,
                           beam_buffer=vals[3] if len(vals) > 3 else 0)
        launch = dict(ann.ann_get_launch(ix, a.mode), tuned_on=None)
    elif not a.no_autotune and not a.headline_only:
        for mode, e_, rr in ((a.mode, ef, a.rerank), ("f32", ef32, 0)):
            t = time.perf_counter()
            best = ann.ann_autotune(ix, mode, queries=Qd[:a.tune_nq], k=k, ef=e_, rerank=rr)
            log(f"autotuned {mode} on {min(a.tune_nq, Q.shape[0])} queries in "
                f"{time.perf_counter() - t:.1f}s: {best}")
            if mode == a.mode:
                launch = dict(best, tuned_on=min(a.tune_nq, Q.shape[0]))
            else:
                launch32 = dict(best, tuned_on=min(a.tune_nq, Q.shape[0]))

    # headline mode
    head = Timed(ann, torch, ix, a.mode, Qd, k, ef, a.rerank, stream)
    ms, wall = head.run(a.steps, a.warmup)
    ids = head.out["ids"].cpu().numpy()
    rec = recall(ids, gt, k) if gt is not None else None
    qps = Q.shape[0] / (ms / 1e3)
    st = head.step(stats=True)
    torch.cuda.synchronize()
    stats = st["stats"].cpu().numpy()
    nbytes = algorithmic_bytes(stats, a.mode, d, g.M0, k, a.rerank)
    achieved = nbytes / (ms / 1e3) / 1e9
    log(f"{a.mode}+rerank{a.rerank} ef={ef}: {ms:.2f} ms/step, {qps:.0f} QPS, recall {rec}, "
        f"{achieved:.0f} GB/s algorithmic")

    if a.headline_only:
        print(json.dumps({"mode": a.mode, "ef": ef, "ms_per_step": round(ms, 3), "qps": round(qps, 1),
                          "recall@10": rec, "algorithmic_bytes_per_launch": nbytes}), flush=True)
        ix.close()
        return

    # FP32 beside it
    f32 = Timed(ann, torch, ix, "f32", Qd, k, ef32, 0, stream)
    ms32, _ = f32.run(a.steps, a.warmup)
    rec32 = recall(f32.out["ids"].cpu().numpy(), gt, k) if gt is not None else None
    st32 = f32.step(stats=True)
    torch.cuda.synchronize()
    b32 = algorithmic_bytes(st32["stats"].cpu().numpy(), "f32", d, g.M0, k, 0)
    log(f"f32 ef={ef32}: {ms32:.2f} ms/step, {Q.shape[0] / (ms32 / 1e3):.0f} QPS, recall {rec32}")

    # one small batch replayed as a captured graph (ann_plan_*) against the
    # same batch launched directly: the host cost of a launch
    captured = None
    try:
        nb_, ef_s = 64, 64
        plan = ann.Plan(ix, a.mode, capacity=nb_, k=k, ef=ef_s, rerank=a.rerank)
        plan.queries.copy_(Qd[:nb_])
        torch.cuda.synchronize()
        reps = 200
        for _ in range(5):
            plan.launch(nb_, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            plan.launch(stream=stream)
        torch.cuda.synchronize()
        t_graph = (time.perf_counter() - t) / reps
        qs = Qd[:nb_]
        out_d = None
        for _ in range(5):
            out_d = ann.ann_search_ex(ix, a.mode, queries=qs, k=k, ef=ef_s, rerank=a.rerank,
                                      stream=stream, out=out_d)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            ann.ann_search_ex(ix, a.mode, queries=qs, k=k, ef=ef_s, rerank=a.rerank,
                              stream=stream, out=out_d)
        torch.cuda.synchronize()
        t_direct = (time.perf_counter() - t) / reps
        same = bool(torch.equal(plan.ids[:nb_], out_d["ids"]))
        captured = {"nq": nb_, "ef": ef_s, "graph_us_per_batch": round(t_graph * 1e6, 1),
                    "direct_us_per_batch": round(t_direct * 1e6, 1), "same_results": same,
                    "launch": plan.info()}
        plan.close()
        log(f"captured batch of {nb_} at ef {ef_s}: {captured}")
    except ann.AnnError as e:
        log(f"captured batch skipped: {e}")

    # BF16 rows + the same rerank (an extra row beside the headline)
    bf16_row = None
    if not a.no_bf16:
        u = X.view(np.uint32)
        xb = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)   # round to nearest even
        ixb = ann.ann_index_create(g, spec["metric"], d, x_f32=X, x_bf16=xb)
        del xb
        if launch:
            ann.ann_set_launch(ixb, "bf16", slots=launch["slots"],
                               lanes_per_row=launch["lanes_per_row"],
                               waves_per_query=launch["waves_per_query"],
                               beam_buffer=launch["beam_buffer"])
        tb = Timed(ann, torch, ixb, "bf16", Qd, k, ef, a.rerank, stream)
        msb, _ = tb.run(min(a.steps, 5), min(a.warmup, 1))
        recb = recall(tb.out["ids"].cpu().numpy(), gt, k) if gt is not None else None
        stb = tb.step(stats=True)
        torch.cuda.synchronize()
        bb = algorithmic_bytes(stb["stats"].cpu().numpy(), "bf16", d, g.M0, k, a.rerank)
        bf16_row = {"ef": ef, "qps": round(Q.shape[0] / (msb / 1e3), 1), "recall@10": recb,
                    "ms_per_step": round(msb, 3), "algorithmic_GBps": round(bb / (msb / 1e3) / 1e9, 1)}
        ixb.close()
        log(f"bf16+rerank{a.rerank} ef={ef}: {msb:.2f} ms/step, {bf16_row['qps']:.0f} QPS, recall {recb}")

    # exact k-NN on matrix cores (ground truth path): one launch, all queries
    bf = bruteforce_row(ann, torch, ix, Qd, k, stream, gt, X.shape[0], d)

    # IVF index over the same rows (an index family beside the graph)
    ivf_rows = None
    if ivf is not None:
        ivf_rows = {"nlist": nlist}
        for key, mode, rr in (("f16+rerank", a.mode, a.rerank), ("f32", "f32", 0)):
            npb, _ = pick_nprobe(ivf_sweep, key)
            if npb is None:
                continue
            traffic = None
            tp = os.path.join(PROFILES, f"ivf_{a.workload}_traffic.json")
            if os.path.exists(tp):
                t = json.load(open(tp))
                if (t.get("nprobe") == npb and t.get("mode") == mode and t.get("rerank") == rr
                        and t.get("kernel_sha") == ivf_sha()):
                    traffic = t.get("bytes_per_launch")
            ivf_rows[key] = ivf_row(ann, torch, ivf, mode, Qd, k, npb, rr, stream, gt, d, nlist,
                                    a.steps, a.warmup, traffic=traffic)
            rf = ivf_rows[key]["roofline"]
            log(f"ivf {key} nprobe={npb}: {ivf_rows[key]['qps']:.0f} QPS, recall "
                f"{ivf_rows[key]['recall@10']}, {rf['achieved']} {rf['unit']} ({rf['bound']}, "
                f"{rf['frac']:.3f} of peak)")
        if ivf_sweep:
            ivf_rows["nprobe_sweep"] = {k_: [[r["nprobe"], round(r["recall"], 4), round(r["qps"], 1)]
                                             for r in v] for k_, v in ivf_sweep.items()
                                        if isinstance(v, list)}

    serve = serve32 = None
    if not a.no_serve:
        try:
            serve = serve_latency(ann, ix, Q, k, ef, a.mode, a.rerank, qps, waves=a.serve_waves)
            log(f"serving {a.mode}: {serve}")
            qps32 = Q.shape[0] / (ms32 / 1e3)
            serve32 = serve_latency(ann, ix, Q, k, ef32, "f32", 0, qps32, waves=a.serve_waves)
            log(f"serving f32: {serve32}")
        except ann.AnnError as e:
            log(f"serving skipped: {e}")

    cpu = cpu1 = cpux = None
    if not a.no_cpu:
        cpu, cpu1, cpux = cpu_baseline(g, X, Q, a.mode, ef, k, a.rerank)
        log(f"cpu oracle: {cpu['value']:.1f} QPS on {cpu['cores']} threads, "
            f"{cpu1['value']:.2f} QPS on one thread, {cpux['value']:.1f} QPS with EXACT keys")

    traffic = None
    tp = os.path.join(PROFILES, f"search_{a.workload}_traffic.json")
    if os.path.exists(tp):
        t = json.load(open(tp))
        shape = None
        if launch:
            shape = ",".join(str(launch[f]) for f in ("slots", "lanes_per_row", "waves_per_query",
                                                      "beam_buffer"))
        # counters describe one kernel version at one launch shape
        if (t.get("ef") == ef and t.get("mode") == a.mode and t.get("kernel_sha") == kernel_sha()
                and t.get("launch") == shape):
            traffic = t.get("bytes_per_launch")

    out = {
        "metric": "QPS at recall@10>=0.95, 1M x 768 HNSW: FP16 traversal + FP32 rerank vs FP32",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded vMF mixture; graph and ground truth from the CPU oracle)",
        "config": {
            "workload": f"{a.workload}: {spec['n']:,} x {d} unit-norm vMF mixture "
                        f"({spec['centres']} clusters, kappa {spec['kappa']}), inner product, "
                        f"HNSW M={spec['M']} efC={spec['efc']}, {Q.shape[0]:,} queries, k={k}",
            "storage": f"{a.mode} rows, fp32 arithmetic, fp32 rerank of {a.rerank}",
            "launch": launch or ann.ann_get_launch(ix, a.mode),
            "captured_batch": captured,
            "ef": ef, "recall@10": rec,
            "recall_target_met": (rec is not None and rec >= 0.95),
            "ef_sweep": ({k_: [[r["ef"], round(r["recall"], 4), round(r["qps"], 1)] for r in v]
                          for k_, v in sweep.items() if isinstance(v, list)} if sweep else None),
            "p50_ms": serve and serve["p50_ms"], "p99_ms": serve and serve["p99_ms"],
            "serving": serve,
            "f32": {"ef": ef32, "qps": round(Q.shape[0] / (ms32 / 1e3), 1), "recall@10": rec32,
                    "ms_per_step": round(ms32, 3),
                    "algorithmic_GBps": round(b32 / (ms32 / 1e3) / 1e9, 1),
                    "p50_ms": serve32 and serve32["p50_ms"], "p99_ms": serve32 and serve32["p99_ms"],
                    "serving": serve32, "launch": launch32},
            "bf16+rerank": bf16_row,
            "cpu_oracle_single_thread": cpu1,
            "cpu_oracle_exact_keys": cpux,
            "wall_s": round(wall, 3),
            "bruteforce_mfma": bf,
            "ivf": ivf_rows,
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_launch": nbytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if ivf is not None:
        ivf.close()
    ix.close()


def build_bench(ann, torch, spec, g, X):
    """The graph built on the device with the stored graph's schedule (2,000
    nodes one at a time, then batches of 2% up to 2,048), timed, and compared
    with the stored graph list by list."""
    import synth
    Xd = torch.from_numpy(X).to("cuda:0")
    u = synth.level_uniforms(0, X.shape[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    b = ann.ann_hnsw_build(Xd, spec["metric"], spec["M"], spec["efc"], u, seq_prefix=2000,
                           batch_frac=0.02, batch_cap=2048)
    dt = time.perf_counter() - t
    same = (b.max_level == g.max_level and b.entry == g.entry
            and bool(np.array_equal(b.levels, g.levels)) and bool(np.array_equal(b.adj0, g.adj0))
            and bool(np.array_equal(b.upper_off, g.upper_off))
            and bool(np.array_equal(b.upper_adj, g.upper_adj)))
    log(f"graph built on the device in {dt:.1f}s, equal to the stored graph: {same}")
    print(json.dumps({"build": spec.get("kind"), "n": int(X.shape[0]), "d": int(X.shape[1]),
                      "M": spec["M"], "efc": spec["efc"], "seconds": round(dt, 2),
                      "equal_to_stored_graph": same}), flush=True)


def kernel_sha(pattern="search_*"):
    """Hash of the kernels' sources (the traffic counters describe one version)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2501_06121_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, pattern))):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def ivf_sha():
    """The IVF scan compiles the search's scoring policies (search_impl.h) into ivf.hip."""
    import hashlib
    return hashlib.sha256((kernel_sha("ivf.hip") + kernel_sha("search_impl.h")).encode()).hexdigest()[:16]


if __name__ == "__main__":
    main()
