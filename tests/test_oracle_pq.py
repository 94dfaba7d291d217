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


# Worked example of the empty-cluster rule (the k-means reading: an empty
# cluster takes the sample point of largest current error, lower position on
# ties, each point at most once per iteration, clusters in ascending order).
# One dimension, six points, three centroids that all start at 0:
#   points        0   0   0  -10  10   30
#   assignment    every point to centroid 0 (all keys tie, lower index wins)
#   errors        0   0   0  100 100  900
# centroid 0 = mean = 30 / 6 = 5; centroid 1 (empty) = the largest error,
# 30 (position 5); centroid 2 (empty) = the next one not yet used: -10 and 10
# tie at 100, the lower position (3) wins, so -10.  A second iteration
# assigns {0, 0, 0, 10} -> 0 (keys 25 vs 100 / 25 vs 400), {30} -> 1,
# {-10} -> 2, giving means 2.5, 30, -10.
RESEED_POINTS = np.array([0.0, 0.0, 0.0, -10.0, 10.0, 30.0], np.float32)
RESEED_AFTER = {1: [5.0, 30.0, -10.0], 2: [2.5, 30.0, -10.0]}


def test_empty_cluster_reseed_worked_example_pq():
    X = RESEED_POINTS[:, None]
    sample = np.arange(6, dtype=np.int64)
    init = np.array([0, 1, 2], np.int64)
    for iters, want in RESEED_AFTER.items():
        cb, it, _ = oracle.pq_train(X, 1, 3, sample, init, max_iter=iters, threads=1)
        assert it == iters
        assert cb[0, :, 0].tolist() == want, (iters, cb[0, :, 0])
    # mistakes the rule excludes give other centroids
    wrong = {"smallest error": [5.0, 0.0, 0.0], "point reused": [5.0, 30.0, 30.0],
             "higher position on ties": [5.0, 30.0, 10.0],
             "clusters in descending order": [5.0, -10.0, 30.0]}
    for name, w in wrong.items():
        assert w != RESEED_AFTER[1], name


def test_empty_cluster_reseed_worked_example_ivf():
    # the coarse quantizer runs the same iteration on whole (here 2-d) rows:
    # the second coordinate is 0, so errors and means are those above
    X = np.stack([RESEED_POINTS, np.zeros(6, np.float32)], axis=1)
    sample = np.arange(6, dtype=np.int64)
    init = np.array([0, 1, 2], np.int64)
    for iters, want in RESEED_AFTER.items():
        cent, it, obj = oracle.ivf_train(X, 3, sample, init, max_iter=iters, threads=1)
        assert it == iters
        assert cent[:, 0].tolist() == want and not cent[:, 1].any()
    # the first assignment's summed error is 0 + 0 + 0 + 100 + 100 + 900
    assert obj[0] == 1100.0


def test_reseed_takes_points_in_decreasing_error_order():
    # four empty clusters out of five: they take the four largest-error points
    # in decreasing error order, each once (errors 1, 4, 9, 16, 25, 36 from 0)
    X = np.array([0, 0, 0, 0, 0, 1, 2, 3, 4, 5, 6], np.float32)[:, None]
    sample = np.arange(11, dtype=np.int64)
    init = np.arange(5, dtype=np.int64)
    cb, it, _ = oracle.pq_train(X, 1, 5, sample, init, max_iter=1, threads=1)
    # centroid 0: the FP64 mean of all eleven points (21 / 11), rounded once
    assert cb[0, :, 0].tolist() == [float(np.float32(21.0 / 11.0)), 6.0, 5.0, 4.0, 3.0]
