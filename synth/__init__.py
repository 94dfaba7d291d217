"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers.  It holds none of the search method's
arithmetic (no distances, no graph, no quantizer), so that both the CPU oracle
and the GPU library can take their inputs from it without sharing any code of
the method itself.

The paper evaluates on SIFT1M (dense, L2, 128-d), MS MARCO passage embeddings
(dense, inner product, 768-d) and a SPLADE sparse version of MS MARCO
(Section 3, Table 1).  None of those datasets is used or recreated here; the
generators below produce stand-ins with the same shapes and measures.

Every workload takes one integer seed.  ``SeedSequence(seed)`` is split into
named child streams (centres, base, queries, levels, pq_sample, arrivals,
ivf_sample),
so that for instance the number of queries never changes the base set.  Large
arrays are drawn in chunks of ``CHUNK`` rows, each chunk from its own
grandchild stream, which makes generation order-independent and parallel.
All draws are float64; vectors are cast to float32 (round to nearest even) at
the very end.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

STREAMS = ("centres", "base", "queries", "levels", "pq_sample", "arrivals", "ivf_sample")
CHUNK = 65536


def stream(seed: int, name: str) -> np.random.SeedSequence:
    """The named child stream of ``SeedSequence(seed)``."""
    idx = STREAMS.index(name)
    root = np.random.SeedSequence(seed)
    return np.random.SeedSequence(entropy=root.entropy, spawn_key=root.spawn_key + (idx,))


def _child(ss: np.random.SeedSequence, i: int) -> np.random.Generator:
    return np.random.default_rng(
        np.random.SeedSequence(entropy=ss.entropy, spawn_key=ss.spawn_key + (i,)))


def _chunked(ss, n, fn, threads=None):
    """Run ``fn(rng, m)`` for each CHUNK-row slice of n rows; concatenate."""
    nch = max(1, math.ceil(n / CHUNK))
    sizes = [min(CHUNK, n - c * CHUNK) for c in range(nch)]
    threads = threads or min(16, os.cpu_count() or 1)

    def run(c):
        return fn(_child(ss, c), sizes[c])

    if nch == 1 or threads == 1:
        parts = [run(c) for c in range(nch)]
    else:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(run, range(nch)))
    return np.concatenate(parts, axis=0) if parts else np.zeros((0,))


# --------------------------------------------------------------------------
# Dense: Gaussian mixture (SIFT-like shape, L2)
# --------------------------------------------------------------------------

def gaussian_centres(seed, n_centres, d):
    rng = np.random.default_rng(stream(seed, "centres"))
    return rng.standard_normal((n_centres, d))


def gaussian_mixture(seed, n, d, n_centres, sigma, which="base", threads=None):
    """n points: centre[U{0..C-1}] + sigma * N(0, I), centres ~ N(0, I)."""
    centres = gaussian_centres(seed, n_centres, d)

    def draw(rng, m):
        lab = rng.integers(0, n_centres, size=m)
        x = centres[lab] + sigma * rng.standard_normal((m, d))
        return x.astype(np.float32)

    out = _chunked(stream(seed, which), n, draw, threads)
    return out.reshape(n, d)


# --------------------------------------------------------------------------
# Dense: von Mises-Fisher mixture on the unit sphere (embedding-like, IP)
# --------------------------------------------------------------------------

def vmf_means(seed, n_centres, d):
    rng = np.random.default_rng(stream(seed, "centres"))
    g = rng.standard_normal((n_centres, d))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _wood_w(rng, kappa, p, m):
    """Component along the mean direction, Wood (1994) rejection sampler."""
    b = (p - 1.0) / (2.0 * kappa + math.sqrt(4.0 * kappa * kappa + (p - 1.0) ** 2))
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + (p - 1.0) * math.log(1.0 - x0 * x0)
    a = (p - 1.0) / 2.0
    w = np.empty(m)
    pending = np.arange(m)
    while pending.size:
        z = rng.beta(a, a, size=pending.size)
        u = rng.random(size=pending.size)
        ww = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        ok = kappa * ww + (p - 1.0) * np.log(1.0 - x0 * ww) - c >= np.log(u)
        w[pending[ok]] = ww[ok]
        pending = pending[~ok]
    return w


def vmf_mixture(seed, n, d, n_centres, kappa, which="base", threads=None):
    """n unit-norm points from a uniform mixture of vMF(mu_c, kappa)."""
    means = vmf_means(seed, n_centres, d)

    def draw(rng, m):
        lab = rng.integers(0, n_centres, size=m)
        mu = means[lab]
        w = _wood_w(rng, kappa, d, m)
        v = rng.standard_normal((m, d))
        v -= np.sum(v * mu, axis=1, keepdims=True) * mu
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        x = w[:, None] * mu + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x.astype(np.float32)

    out = _chunked(stream(seed, which), n, draw, threads)
    return out.reshape(n, d)


# --------------------------------------------------------------------------
# Sparse: Zipf term ids, log-normal weights (SPLADE-like shape, IP)
# --------------------------------------------------------------------------

def _first_distinct(D, nnz, vocab):
    """Per row of D (-1 = invalid draw): the first nnz[r] distinct valid values
    in draw order, returned id-sorted and padded with `vocab`; and whether the
    row had enough."""
    m, w = D.shape
    order = np.argsort(D, axis=1, kind="stable")
    S = np.take_along_axis(D, order, axis=1)
    first_sorted = np.ones_like(S, dtype=bool)
    first_sorted[:, 1:] = S[:, 1:] != S[:, :-1]
    first_sorted &= S >= 0
    F = np.zeros_like(first_sorted)
    np.put_along_axis(F, order, first_sorted, axis=1)
    C = np.cumsum(F, axis=1)
    keep = F & (C <= nnz[:, None])
    out = np.where(keep, D, vocab)
    out.sort(axis=1)
    return out, C[:, -1] >= nnz


def _zipf_rows(rng, m, mean_extra, vocab, zipf_a, sigma):
    """m sparse rows; nnz = 1 + Poisson(mean_extra), ids distinct, id-sorted.

    Each row takes, in draw order, the first nnz distinct ids among draws of
    Zipf(zipf_a) truncated to the vocabulary (rank r -> id r - 1).  Draws are
    made in blocks of columns; rows that are still short draw another block.
    """
    nnz = np.minimum(1 + rng.poisson(mean_extra, size=m), vocab)
    width = int(4 * nnz.max()) + 16 if m else 1
    D = rng.zipf(zipf_a, size=(m, width))
    D = np.where(D <= vocab, D - 1, -1).astype(np.int64)
    best, ok = _first_distinct(D, nnz, vocab)
    short = np.flatnonzero(~ok)
    while short.size:
        more = rng.zipf(zipf_a, size=(short.size, width))
        more = np.where(more <= vocab, more - 1, -1).astype(np.int64)
        Ds = np.concatenate([D[short], more], axis=1)
        b2, ok2 = _first_distinct(Ds, nnz[short], vocab)
        cols = min(best.shape[1], b2.shape[1])
        best[short, :cols] = b2[:, :cols]
        D = np.pad(D, ((0, 0), (0, width)), constant_values=-1)
        D[short] = Ds
        short = short[~ok2]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(nnz, out=indptr[1:])
    take = np.arange(best.shape[1])[None, :] < nnz[:, None]
    ids = best[take].astype(np.uint16)
    vals = np.exp(sigma * rng.standard_normal(int(indptr[-1]))).astype(np.float32)
    return indptr, ids, vals


def sparse_zipf(seed, n, mean_nnz, vocab=30522, zipf_a=1.1, sigma=0.5,
                which="base", threads=None):
    """CSR (indptr i64[n+1], ids u16, vals f32) rows with ~mean_nnz nonzeros."""
    ss = stream(seed, which)
    nch = max(1, math.ceil(n / CHUNK))
    sizes = [min(CHUNK, n - c * CHUNK) for c in range(nch)]
    threads = threads or min(16, os.cpu_count() or 1)

    def run(c):
        return _zipf_rows(_child(ss, c), sizes[c], mean_nnz - 1, vocab, zipf_a, sigma)

    if nch == 1 or threads == 1:
        parts = [run(c) for c in range(nch)]
    else:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(run, range(nch)))
    indptr = [np.zeros(1, dtype=np.int64)]
    off = 0
    for ip, _, _ in parts:
        indptr.append(ip[1:] + off)
        off += int(ip[-1])
    return (np.concatenate(indptr), np.concatenate([p[1] for p in parts]),
            np.concatenate([p[2] for p in parts]))


# --------------------------------------------------------------------------
# Random numbers the index construction consumes
# --------------------------------------------------------------------------

def level_uniforms(seed, n):
    """u_i ~ U[0, 1) per base point, consumed by the HNSW level draw."""
    return np.random.default_rng(stream(seed, "levels")).random(n)


def pq_sample(seed, n, n_sample, n_centroids):
    """Training sample ids (without replacement) and the k-means init order.

    Returns (sample_ids i64[n_sample], init i64[n_centroids]) where ``init``
    indexes into the sample: the first n_centroids of a seeded permutation.
    """
    rng = np.random.default_rng(stream(seed, "pq_sample"))
    ids = np.sort(rng.choice(n, size=min(n, n_sample), replace=False)).astype(np.int64)
    init = rng.permutation(ids.size)[:n_centroids].astype(np.int64)
    return ids, init


def ivf_sample(seed, n, n_sample, nlist):
    """Coarse-quantizer training sample ids (without replacement, ascending)
    and the k-means init order (indexes into the sample), like pq_sample but
    from a stream of its own."""
    rng = np.random.default_rng(stream(seed, "ivf_sample"))
    ids = np.sort(rng.choice(n, size=min(n, n_sample), replace=False)).astype(np.int64)
    init = rng.permutation(ids.size)[:nlist].astype(np.int64)
    return ids, init


# --------------------------------------------------------------------------
# Request streams for the serving workload
# --------------------------------------------------------------------------

def arrivals(seed, n_req, rate_qps, k_choices=(10, 100), ef_choices=(64, 128, 256, 512),
             n_pool=None):
    """Poisson arrivals: (t_arrive_s f64, query idx i64, k i32, ef i32)."""
    rng = np.random.default_rng(stream(seed, "arrivals"))
    gaps = rng.exponential(1.0 / rate_qps, size=n_req)
    t = np.cumsum(gaps)
    qidx = rng.integers(0, n_pool or n_req, size=n_req).astype(np.int64)
    k = rng.choice(np.asarray(k_choices, dtype=np.int32), size=n_req)
    ef = rng.choice(np.asarray(ef_choices, dtype=np.int32), size=n_req)
    return t, qidx, k.astype(np.int32), ef.astype(np.int32)


# --------------------------------------------------------------------------
# The named workloads (sizes and distributions of the benchmark configs)
# --------------------------------------------------------------------------

WORKLOADS = {
    # 10k x 128 Gaussian mixture, L2, M=16, efC=100, ef=64, k=10
    "gmm10k": dict(kind="gmm", n=10_000, nq=100, d=128, centres=32, sigma=0.3,
                   metric="l2", M=16, efc=100, ef=64, k=10),
    # 1M x 768 unit-norm vMF mixture, inner product, M=32
    "vmf1m": dict(kind="vmf", n=1_000_000, nq=10_000, d=768, centres=1024, kappa=50.0,
                  metric="ip", M=32, efc=200, ef=128, k=10),
    # 1M sparse docs over 30,522 terms, inner product, M=32
    "splade1m": dict(kind="sparse", n=1_000_000, nq=10_000, vocab=30522, nnz_doc=120,
                     nnz_query=40, metric="ip", M=32, efc=200, ef=100, k=10),
    # 10M x 96 Gaussian mixture, L2, M=32 (serving mix)
    "gmm10m": dict(kind="gmm", n=10_000_000, nq=10_000, d=96, centres=4096, sigma=0.3,
                   metric="l2", M=32, efc=200, ef=128, k=10),
}


def dense_base(spec, seed=0, n=None, threads=None):
    n = spec["n"] if n is None else n
    if spec["kind"] == "gmm":
        return gaussian_mixture(seed, n, spec["d"], spec["centres"], spec["sigma"], "base", threads)
    if spec["kind"] == "vmf":
        return vmf_mixture(seed, n, spec["d"], spec["centres"], spec["kappa"], "base", threads)
    raise ValueError(spec["kind"])


def dense_queries(spec, seed=0, nq=None, threads=None):
    nq = spec["nq"] if nq is None else nq
    if spec["kind"] == "gmm":
        return gaussian_mixture(seed, nq, spec["d"], spec["centres"], spec["sigma"], "queries", threads)
    if spec["kind"] == "vmf":
        return vmf_mixture(seed, nq, spec["d"], spec["centres"], spec["kappa"], "queries", threads)
    raise ValueError(spec["kind"])
