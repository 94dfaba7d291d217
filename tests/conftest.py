"""Shared fixtures: small seeded workloads built by the CPU oracle."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def gmm10k():
    """10,000 x 128 Gaussian mixture, 100 queries, L2, M=16, efC=100 (sequential build)."""
    spec = synth.WORKLOADS["gmm10k"]
    X = synth.dense_base(spec)
    Q = synth.dense_queries(spec)
    u = synth.level_uniforms(0, X.shape[0])
    g = oracle.hnsw_build(X, "l2", spec["M"], spec["efc"], u)
    return dict(spec=spec, X=X, Q=Q, graph=g, metric="l2")


@pytest.fixture(scope="session")
def vmf_small():
    """4,096 x 768 unit-norm vMF mixture (kappa 50), 64 queries, IP, M=32, efC=100."""
    spec = synth.WORKLOADS["vmf1m"]
    n = 4096
    X = synth.dense_base(spec, n=n)
    Q = synth.dense_queries(spec, nq=64)
    u = synth.level_uniforms(0, n)
    g = oracle.hnsw_build(X, "ip", 32, 100, u, seq_prefix=1000, batch_frac=0.02, batch_cap=256)
    return dict(spec=spec, X=X, Q=Q, graph=g, metric="ip")


@pytest.fixture(scope="session")
def sparse_small():
    """3,000 sparse docs over 2,000 terms (~30 nnz), 48 queries (~10 nnz), IP, M=16."""
    n, vocab = 3000, 2000
    ip, ids, vals = synth.sparse_zipf(7, n, 30, vocab=vocab, which="base")
    qp, qi, qv = synth.sparse_zipf(7, 48, 10, vocab=vocab, which="queries")
    st = oracle.sparse_store(ip, ids, vals, vocab)
    g = oracle.hnsw_build_sparse(ip, ids, vals, vocab, 16, 64, synth.level_uniforms(7, n))
    return dict(indptr=ip, ids=ids, vals=vals, q=(qp, qi, qv), vocab=vocab, store=st, graph=g)


def small_int_points(seed, n, d, lo=-4, hi=5):
    """Integer coordinates: every FP32 product and sum below 2^24 is exact."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(n, d)).astype(np.float32)
