"""Product Quantization on the device (training and encoding) against the
oracle, bit for bit: codes, codebooks and iteration counts."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-pq]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def train_both(X, m, ksub, n_sample, max_iter, seed=0):
    sample, init = synth.pq_sample(seed, X.shape[0], n_sample, ksub)
    ref_cb, ref_it, _ = oracle.pq_train(X, m, ksub, sample, init, max_iter)
    cb, it = ann.ann_pq_train(dev(X), dev(sample), dev(init), m, ksub, max_iter)
    torch.cuda.synchronize()
    return cb.cpu().numpy(), it, ref_cb, ref_it


def test_train_and_encode_gmm10k(gmm10k):
    X = gmm10k["X"]
    say("train 16 x 256 on 5,000 of 10,000 x 128")
    cb, it, ref_cb, ref_it = train_both(X, 16, 256, 5000, 8)
    assert it == ref_it
    assert np.array_equal(cb.view(np.uint32), ref_cb.view(np.uint32))
    say("encode 10,000 rows")
    codes = ann.ann_pq_encode(dev(X), dev(ref_cb)).cpu().numpy()
    assert np.array_equal(codes, oracle.pq_encode(X, ref_cb))


def test_train_and_encode_768(vmf_small):
    X = vmf_small["X"]
    say("train 64 x 256 (12 dimensions each) on 4,096 x 768")
    cb, it, ref_cb, ref_it = train_both(X, 64, 256, X.shape[0], 6)
    assert it == ref_it
    assert np.array_equal(cb.view(np.uint32), ref_cb.view(np.uint32))
    codes = ann.ann_pq_encode(dev(X), dev(ref_cb)).cpu().numpy()
    assert np.array_equal(codes, oracle.pq_encode(X, ref_cb))


def test_empty_clusters_and_ties():
    """40 distinct rows repeated 50 times for 256 centroids: most clusters
    empty after the first assignment (re-seeded by error order), exact ties
    everywhere (lower index wins), and convergence before max_iter."""
    rng = np.random.default_rng(5)
    base = rng.standard_normal((40, 32)).astype(np.float32)
    X = np.tile(base, (50, 1))
    say("empty clusters: 2,000 rows, 40 distinct")
    cb, it, ref_cb, ref_it = train_both(X, 4, 256, 2000, 10, seed=3)
    assert it == ref_it
    assert np.array_equal(cb.view(np.uint32), ref_cb.view(np.uint32))
    codes = ann.ann_pq_encode(dev(X), dev(ref_cb)).cpu().numpy()
    assert np.array_equal(codes, oracle.pq_encode(X, ref_cb))


def test_small_codebooks_and_ragged_rows():
    """ksub below 256, subspaces of 1 and of 32 dimensions, n not a multiple
    of the 256-point block."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((1000 + 13, 64)).astype(np.float32)
    for m, ksub in ((64, 16), (2, 64)):
        say("m", m, "ksub", ksub)
        cb, it, ref_cb, ref_it = train_both(X, m, ksub, 700, 5, seed=m)
        assert it == ref_it
        assert np.array_equal(cb.view(np.uint32), ref_cb.view(np.uint32))
        codes = ann.ann_pq_encode(dev(X), dev(ref_cb)).cpu().numpy()
        assert np.array_equal(codes, oracle.pq_encode(X, ref_cb))


def test_empty_cluster_reseed_worked_example():
    """The hand-worked re-seed case of the CPU pins (one dimension, points
    0 0 0 -10 10 30, three centroids at 0): after one iteration 5, 30, -10;
    after two 2.5, 30, -10."""
    X = np.array([0.0, 0.0, 0.0, -10.0, 10.0, 30.0], np.float32)[:, None]
    for iters, want in {1: [5.0, 30.0, -10.0], 2: [2.5, 30.0, -10.0]}.items():
        cb, it = ann.ann_pq_train(dev(X), dev(np.arange(6, dtype=np.int64)),
                                  dev(np.array([0, 1, 2], np.int64)), 1, 3, iters)
        torch.cuda.synchronize()
        assert it == iters
        assert cb.cpu().numpy()[0, :, 0].tolist() == want
