"""Pins of the oracle's keys: closed forms, exact small-integer cases, bounds."""
import numpy as np
import pytest

import oracle
from conftest import small_int_points


def _rows(n, per, nq, seed=0):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=(nq, per)).astype(np.int64)


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("d", [16, 96, 128, 768, 784])
def test_canon_exact_on_small_integers(metric, d):
    # integer coordinates: every product and partial sum is exact in FP32,
    # so any evaluation order gives the exact integer key
    X = small_int_points(1, 300, d)
    Q = small_int_points(2, 20, d)
    st = oracle.dense_store(X, metric)
    rows = _rows(300, 40, 20)
    canon = oracle.keys(st, Q, rows, "canon")
    exact = oracle.keys(st, Q, rows, "exact")
    Xi = X.astype(np.int64); Qi = Q.astype(np.int64)
    if metric == "ip":
        ref = -np.einsum("qd,qkd->qk", Qi, Xi[rows])
    else:
        ref = ((Qi[:, None, :] - Xi[rows]) ** 2).sum(-1)
    assert np.array_equal(canon, ref.astype(np.float32))
    assert np.array_equal(exact, ref.astype(np.float32))


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_canon_within_error_bound(metric):
    rng = np.random.default_rng(3)
    d = 768
    X = rng.standard_normal((500, d)).astype(np.float32)
    Q = rng.standard_normal((16, d)).astype(np.float32)
    st = oracle.dense_store(X, metric)
    rows = _rows(500, 100, 16)
    canon = oracle.keys(st, Q, rows, "canon").astype(np.float64)
    Qd = Q.astype(np.float64); Xd = X.astype(np.float64)[rows]
    if metric == "ip":
        terms = Qd[:, None, :] * Xd
        ref = -terms.sum(-1)
    else:
        terms = (Qd[:, None, :] - Xd) ** 2
        ref = terms.sum(-1)
    mag = np.abs(terms).sum(-1)
    # each partial: ceil(d/256)*4 fmas; then 6 tree adds: (d/64 + 6 + 2) ulps
    bound = (d / 64 + 6 + 2) * 2.0 ** -24 * mag
    assert np.all(np.abs(canon - ref) <= bound)
    assert np.all(np.abs(canon - ref) <= 1e-5 * np.maximum(np.abs(ref), mag))
    exact = oracle.keys(st, Q, rows, "exact").astype(np.float64)
    assert np.all(np.abs(exact - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-30)


def test_ip_key_is_negated_dot_and_l2_is_squared():
    X = np.float32([[1, 2, 3, 4] * 4])
    Q = np.float32([[2, 0, 1, 0] * 4])
    assert oracle.keys(oracle.dense_store(X, "ip"), Q, [[0]], "canon")[0, 0] == -20.0
    assert oracle.keys(oracle.dense_store(X, "l2"), Q, [[0]], "canon")[0, 0] == 4 * (1 + 4 + 4 + 16)


@pytest.mark.parametrize("mode", ["f16", "bf16", "fp8"])
@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_reduced_precision_keys_use_the_decoded_vector(mode, metric):
    rng = np.random.default_rng(4)
    d = 128
    X = (rng.standard_normal((200, d)) * 0.05).astype(np.float32)
    Q = (rng.standard_normal((8, d)) * 0.05).astype(np.float32)
    if mode == "f16":
        codes, scale = oracle.to_f16(X), None
        dec = oracle.from_f16(codes)
    elif mode == "bf16":
        codes, scale = oracle.to_bf16(X), None
        dec = oracle.from_bf16(codes)
    else:
        codes, scale = oracle.encode_fp8_rows(X)
        dec = oracle.from_e4m3(codes).astype(np.float64) * scale[:, None].astype(np.float64)
    st = oracle.dense_store(codes, metric, mode, fp8_scale=scale)
    rows = _rows(200, 30, 8)
    exact = oracle.keys(st, Q, rows, "exact").astype(np.float64)
    canon = oracle.keys(st, Q, rows, "canon").astype(np.float64)
    Dd = np.asarray(dec, np.float64)[rows]
    Qd = Q.astype(np.float64)[:, None, :]
    terms = Qd * Dd if metric == "ip" else (Qd - Dd) ** 2
    ref = -terms.sum(-1) if metric == "ip" else terms.sum(-1)
    mag = np.abs(terms).sum(-1)
    assert np.all(np.abs(exact - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30)
    tol = 1e-5 * np.maximum(np.abs(ref), mag)
    if mode == "fp8" and metric == "l2":
        tol = tol + 4 * 2.0 ** -24 * mag  # extra rounding of scale * x
    assert np.all(np.abs(canon - ref) <= tol)


def test_sparse_equals_densified_dot():
    import synth
    ip, ids, vals = synth.sparse_zipf(3, 200, 30, vocab=1000)
    qp, qi, qv = synth.sparse_zipf(3, 10, 12, vocab=1000, which="queries")
    st = oracle.sparse_store(ip, ids, vals, 1000)
    D = np.zeros((200, 1000)); Qd = np.zeros((10, 1000))
    for r in range(200):
        D[r, ids[ip[r]:ip[r + 1]]] = vals[ip[r]:ip[r + 1]]
    for r in range(10):
        Qd[r, qi[qp[r]:qp[r + 1]]] = qv[qp[r]:qp[r + 1]]
    rows = np.tile(np.arange(200), (10, 1))
    ref = -(Qd @ D.T)
    exact = oracle.keys(st, None, rows, "exact", sparse_q=(qp, qi, qv)).astype(np.float64)
    canon = oracle.keys(st, None, rows, "canon", sparse_q=(qp, qi, qv)).astype(np.float64)
    assert np.all(np.abs(exact - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-30)
    assert np.all(np.abs(canon - ref) <= 1e-5 * np.abs(ref) + 1e-30)
    disjoint = ref == 0
    assert np.all(canon[disjoint] == 0)
    # symmetric: doc 5 as query against doc 9 and vice versa
    sym_q = (np.array([0, ip[6] - ip[5]]), ids[ip[5]:ip[6]], vals[ip[5]:ip[6]])
    sym_q2 = (np.array([0, ip[10] - ip[9]]), ids[ip[9]:ip[10]], vals[ip[9]:ip[10]])
    a = oracle.keys(st, None, [[9]], "exact", sparse_q=sym_q)
    b = oracle.keys(st, None, [[5]], "exact", sparse_q=sym_q2)
    assert a[0, 0] == b[0, 0]


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_adc_equals_key_of_reconstruction(metric):
    rng = np.random.default_rng(5)
    n, d, m = 300, 96, 8
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((6, d)).astype(np.float32)
    cb = rng.standard_normal((m, 256, d // m)).astype(np.float32)
    codes = oracle.pq_encode(X, cb)
    st = oracle.pq_store(cb, codes, metric)
    rec = np.concatenate([cb[s][codes[:, s]] for s in range(m)], axis=1).astype(np.float64)
    Qd = Q.astype(np.float64)
    ref = -(Qd @ rec.T) if metric == "ip" else ((Qd[:, None, :] - rec[None]) ** 2).sum(-1)
    rows = np.tile(np.arange(n), (6, 1))
    exact = oracle.keys(st, Q, rows, "exact").astype(np.float64)
    canon = oracle.keys(st, Q, rows, "canon").astype(np.float64)
    assert np.allclose(exact, ref, rtol=1e-6, atol=1e-6)
    terms = np.abs(Qd[:, None, :] * rec[None]).sum(-1) if metric == "ip" else np.abs(ref)
    assert np.all(np.abs(canon - ref) <= 1e-5 * np.maximum(np.abs(ref), terms))
    # the tables themselves: per-subspace partial keys
    lut = oracle.pq_luts(st, Q, "exact").astype(np.float64)
    for s in range(m):
        sub = Qd[:, s * 12:(s + 1) * 12]
        c = cb[s].astype(np.float64)
        ref_lut = sub @ c.T if metric == "ip" else ((sub[:, None, :] - c[None]) ** 2).sum(-1)
        assert np.allclose(lut[:, s], ref_lut, rtol=1e-6, atol=1e-6)
