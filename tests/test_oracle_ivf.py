"""Pins of the oracle's IVF index: coarse k-means, list assignment and the
probe-and-scan search, each checked against something other than itself
(closed forms, NumPy brute force in FP64, the oracle's independent full scan)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _data(seed=0, n=3000, d=32, centres=24, nlist=16, nq=20):
    X = synth.gaussian_mixture(seed, n, d, centres, 0.4)
    Q = synth.gaussian_mixture(seed, nq, d, centres, 0.4, "queries")
    sample, init = synth.ivf_sample(seed, n, 1500, nlist)
    cent, iters, obj = oracle.ivf_train(X, nlist, sample, init, max_iter=20)
    asg = oracle.ivf_assign(X, cent)
    off, ids = oracle.ivf_lists(asg, nlist)
    return X, Q, cent, asg, off, ids


def test_single_list_centroid_is_the_mean():
    # one centroid: Lloyd converges at once to the FP64 mean of the sample
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 16)).astype(np.float32)
    sample = np.arange(0, 500, 2, dtype=np.int64)
    cent, iters, _ = oracle.ivf_train(X, 1, sample, np.array([7]), max_iter=5)
    want = np.array([math.fsum(X[sample, t].astype(np.float64)) / sample.size for t in range(16)])
    assert iters == 2   # the first assignment changes, the second does not
    assert np.all(np.abs(cent[0].astype(np.float64) - want) <= np.spacing(np.abs(want).astype(np.float32)))


def test_planted_clusters_are_recovered():
    # 8 far-apart blobs, one initial centroid in each: the centroids become
    # the blob means and every point lands in its own blob's list
    rng = np.random.default_rng(4)
    centres = rng.standard_normal((8, 12)) * 50
    lab = np.repeat(np.arange(8), 60)
    X = (centres[lab] + rng.standard_normal((480, 12))).astype(np.float32)
    sample = np.arange(480, dtype=np.int64)
    init = np.arange(8, dtype=np.int64) * 60 + 5
    cent, iters, obj = oracle.ivf_train(X, 8, sample, init, max_iter=10)
    for c in range(8):
        m = X[lab == c].astype(np.float64).mean(0)
        assert np.allclose(cent[c], m, atol=1e-5)
    assert np.array_equal(oracle.ivf_assign(X, cent), lab)
    assert iters == 2 and obj[1] <= obj[0]


def test_objective_non_increasing():
    X = synth.gaussian_mixture(5, 4000, 24, 32, 0.5)
    sample, init = synth.ivf_sample(5, 4000, 3000, 64)
    _, iters, obj = oracle.ivf_train(X, 64, sample, init, max_iter=15)
    o = obj[:iters]
    assert np.all(o[1:] <= o[:-1] * (1 + 1e-9))


def test_assignment_is_fp64_argmin_and_lists_partition():
    X, _, cent, asg, off, ids = _data()
    d2 = ((X.astype(np.float64)[:, None, :] - cent.astype(np.float64)[None]) ** 2).sum(-1)
    assert np.array_equal(asg, d2.argmin(1))
    assert off[0] == 0 and off[-1] == X.shape[0] and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(X.shape[0]))
    for l in range(cent.shape[0]):
        seg = ids[off[l]:off[l + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(asg[seg] == l)


@pytest.mark.parametrize("mode", ["f32", "f16"])
@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_all_lists_probed_equals_full_scan(mode, metric):
    # nprobe = nlist scans every row once: the result is the oracle's
    # independent brute force with the same keys
    X, Q, cent, _, off, ids = _data(seed=1)
    st = oracle.dense_store(X if mode == "f32" else oracle.to_f16(X), metric, mode)
    r = oracle.ivf_search(st, cent, off, ids, Q, 10, cent.shape[0])
    bi, bk = oracle.bruteforce(st, X.shape[0], 10, Q=Q, kmode="canon")
    assert np.array_equal(r["ids"], bi) and np.array_equal(r["keys"], bk)
    assert np.all(r["stats"][:, 0] == X.shape[0]) and np.all(r["stats"][:, 1] == cent.shape[0])


def test_probes_and_candidates_match_fp64_reference():
    X, Q, cent, _, off, ids = _data(seed=2)
    nprobe = 3
    st = oracle.dense_store(X, "l2")
    r = oracle.ivf_search(st, cent, off, ids, Q, 10, nprobe, w_cap=X.shape[0])
    X64, C64 = X.astype(np.float64), cent.astype(np.float64)
    for i, q in enumerate(Q.astype(np.float64)):
        pk = ((C64 - q) ** 2).sum(1)
        order = np.argsort(pk, kind="stable")
        gaps = np.diff(pk[order])[:nprobe]
        assert gaps.min() > 1e-4 * pk.max()   # no near-tie at the cut (the draw has none)
        assert np.array_equal(r["probes"][i], order[:nprobe])
        cand = np.concatenate([ids[off[l]:off[l + 1]] for l in order[:nprobe]])
        assert r["stats"][i, 0] == cand.size
        w = r["w_ids"][i][:cand.size]
        assert np.array_equal(np.sort(w), np.sort(cand)) and np.all(r["w_ids"][i][cand.size:] == -1)
        # candidates ascend by FP64 key except within the FP32 rounding
        k64 = ((X64[w] - q) ** 2).sum(1)
        assert np.all(np.diff(k64) >= -1e-5 * k64.max())
        # the top 10 are the FP64 top 10 of the candidates
        best = cand[np.argsort(((X64[cand] - q) ** 2).sum(1), kind="stable")[:10]]
        assert set(r["ids"][i].tolist()) == set(best.tolist())


def test_rerank_over_everything_is_the_fp32_scan():
    # F16 scan, rerank depth >= n over all lists: the FP32 keys decide alone
    X, Q, cent, _, off, ids = _data(seed=3, n=800)
    st = oracle.dense_store(oracle.to_f16(X), "ip", "f16")
    r = oracle.ivf_search(st, cent, off, ids, Q, 10, cent.shape[0], rerank_f32=X, rerank_depth=800)
    bi, bk = oracle.bruteforce(oracle.dense_store(X, "ip"), 800, 10, Q=Q, kmode="canon")
    assert np.array_equal(r["ids"], bi) and np.array_equal(r["keys"], bk)


def test_fewer_candidates_than_k_pad():
    # three rows in one list, the rest elsewhere: one probe of that list
    # yields three results and -1 / +inf padding
    X = np.array([[0, 0], [0.1, 0], [0, 0.1], [9, 9], [9.1, 9], [9, 9.1], [9.2, 9]], np.float32)
    X = np.pad(X, ((0, 0), (0, 2)))
    cent = np.array([[0, 0, 0, 0], [9, 9, 0, 0]], np.float32)
    off, ids = oracle.ivf_lists(oracle.ivf_assign(X, cent), 2)
    assert off.tolist() == [0, 3, 7]
    r = oracle.ivf_search(oracle.dense_store(X, "l2"), cent, off, ids, np.zeros((1, 4), np.float32), 5, 1)
    assert r["ids"][0].tolist() == [0, 1, 2, -1, -1]
    assert np.isinf(r["keys"][0, 3:]).all() and r["keys"][0, 0] == 0.0
    assert r["probes"][0].tolist() == [0]
    r = oracle.ivf_search(oracle.dense_store(X, "l2"), cent, off, ids, np.zeros((1, 4), np.float32), 2, 5)
    assert r["probes"][0].tolist() == [0, 1, -1, -1, -1] and r["stats"][0].tolist() == [7, 2]
