"""Distance error of the reduced-precision storage formats against FP64.

Test infrastructure (oracle only).  For the final beams W of 1,000 queries
(FP32 search, ef = 100) on a workload's oracle-built graph, every entry's key
is evaluated in each storage format with the fixed FP32 order the GPU uses
(CANON) and compared with the FP64 key of the FP32 originals (EXACT):
|key_format - key_fp64| / sum_i |q_i x_i|, max and mean per format.

Usage: python -m oracle.format_error vmf1m [--nq 1000] [--ef 100]
Writes profiles/<workload>_format_error.json and prints a markdown table.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--nq", type=int, default=1000)
    ap.add_argument("--ef", type=int, default=100)
    a = ap.parse_args(argv)
    spec = synth.WORKLOADS[a.workload]
    g = oracle.Graph.load(os.path.join(ROOT, "data", a.workload, "graph.npz"))
    X = synth.dense_base(spec)
    Q = synth.dense_queries(spec, nq=a.nq)
    metric = spec["metric"]
    r = oracle.hnsw_search(g, oracle.dense_store(X, metric), 10, a.ef, Q=Q, want_w=True)
    rows = r["w_ids"].astype(np.int64)
    assert (rows >= 0).all()
    exact = oracle.keys(oracle.dense_store(X, metric), Q, rows, "exact").astype(np.float64)
    # sum |q_i x_i| (IP) or sum (q_i - x_i)^2 (L2) in FP64
    Xr = X[rows].astype(np.float64)
    Qd = Q.astype(np.float64)[:, None, :]
    mag = np.abs(Qd * Xr).sum(-1) if metric == "ip" else ((Qd - Xr) ** 2).sum(-1)
    f8, s8 = oracle.encode_fp8_rows(X)
    stores = {
        "f32": oracle.dense_store(X, metric),
        "f16": oracle.dense_store(oracle.to_f16(X), metric, "f16"),
        "bf16": oracle.dense_store(oracle.to_bf16(X), metric, "bf16"),
        "fp8-e4m3+scale": oracle.dense_store(f8, metric, "fp8", fp8_scale=s8),
    }
    out = {"workload": a.workload, "queries": a.nq, "ef": a.ef, "entries": int(rows.size),
           "measure": "|key - key_fp64| / sum|q_i x_i| over the final beams", "formats": {}}
    print("| format | max rel. error | mean rel. error |")
    print("|---|---|---|")
    for name, st in stores.items():
        kk = oracle.keys(st, Q, rows, "canon").astype(np.float64)
        rel = np.abs(kk - exact) / mag
        out["formats"][name] = {"max": float(rel.max()), "mean": float(rel.mean())}
        print(f"| {name} | {rel.max():.3e} | {rel.mean():.3e} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{a.workload}_format_error.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
