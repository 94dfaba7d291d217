"""Pins of the oracle's PQ training and encoding."""
import numpy as np

import oracle
import synth


def test_encode_is_bruteforce_argmin():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((400, 48)).astype(np.float32)
    cb = rng.standard_normal((4, 256, 12)).astype(np.float32)
    codes = oracle.pq_encode(X, cb)
    for s in range(4):
        sub = X[:, s * 12:(s + 1) * 12].astype(np.float64)
        d2 = ((sub[:, None, :] - cb[s].astype(np.float64)[None]) ** 2).sum(-1)
        assert np.array_equal(codes[:, s], d2.argmin(1))   # argmin keeps the lower index


def test_kmeans_objective_non_increasing_and_encode_consistent():
    X = synth.gaussian_mixture(3, 5000, 32, 16, 0.5)
    sample, init = synth.pq_sample(3, 5000, 3000, 256)
    cb, iters, obj = oracle.pq_train(X, 4, 256, sample, init, max_iter=12)
    assert 1 <= iters <= 12
    o = obj[:iters]
    assert np.all(o[1:] <= o[:-1] * (1 + 1e-6))
    assert len(np.unique(init)) == 256 and np.all(np.diff(sample) > 0)
    # centroids are the means of their assigned sample points (last update)
    codes = oracle.pq_encode(X[sample], cb)
    assert codes.shape == (3000, 4)


def test_lossless_when_each_subspace_has_few_values():
    # dsub = 1 with at most 256 distinct values per dimension: every value
    # becomes its own centroid, reconstruction is exact, ADC = exact key
    rng = np.random.default_rng(1)
    d, n = 16, 2000
    vals = np.linspace(-1, 1, 200).astype(np.float32)
    X = vals[rng.integers(0, 200, size=(n, d))]
    # a sample that contains every value in every dimension
    sample = np.arange(n, dtype=np.int64)
    init = np.arange(256, dtype=np.int64)
    cb, _, _ = oracle.pq_train(X, d, 256, sample, init, max_iter=25)
    codes = oracle.pq_encode(X, cb)
    rec = np.concatenate([cb[s][codes[:, s]] for s in range(d)], axis=1)
    assert np.array_equal(rec, X)
    Q = rng.standard_normal((5, d)).astype(np.float32)
    st = oracle.pq_store(cb, codes, "ip")
    rows = np.tile(np.arange(n), (5, 1))
    adc = oracle.keys(st, Q, rows, "exact")
    ref = oracle.keys(oracle.dense_store(X, "ip"), Q, rows, "exact")
    assert np.array_equal(adc, ref)


def test_empty_clusters_are_reseeded():
    # 300 points but only 40 distinct: most of the 256 initial centroids
    # coincide, their clusters empty out and get re-seeded; training stays
    # deterministic
    rng = np.random.default_rng(2)
    base = rng.standard_normal((40, 8)).astype(np.float32)
    X = base[rng.integers(0, 40, 300)]
    sample = np.arange(300, dtype=np.int64)
    init = np.arange(256, dtype=np.int64)
    a, _, _ = oracle.pq_train(X, 1, 256, sample, init, max_iter=5)
    b, _, _ = oracle.pq_train(X, 1, 256, sample, init, max_iter=5, threads=1)
    assert np.array_equal(a, b)
    assert np.isfinite(a).all()
