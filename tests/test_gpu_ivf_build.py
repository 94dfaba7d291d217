"""GPU parity of the IVF construction: coarse k-means and list assignment on
the device against the oracle's, bit for bit (FP64 distances in the same
order, first minimum, FP64 means in sample order, the same re-seeding)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-ivf-build]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("n,d,nlist,ns,iters", [(10_000, 128, 64, 5000, 25), (4096, 768, 40, 2000, 6),
                                                (3000, 20, 100, 1000, 10), (500, 4, 3, 500, 25)])
def test_train_and_assign_equal_the_oracle(n, d, nlist, ns, iters):
    X = synth.gaussian_mixture(11, n, d, max(4, nlist // 2), 0.4)
    sample, init = synth.ivf_sample(11, n, ns, nlist)
    say(f"n={n} d={d} nlist={nlist} sample={ns} max_iter={iters}")
    ref_c, ref_it, _ = oracle.ivf_train(X, nlist, sample, init, max_iter=iters)
    Xd = dev(X)
    cent, it = ann.ann_ivf_train(Xd, dev(sample), dev(init), nlist, max_iter=iters)
    torch.cuda.synchronize()
    assert it == ref_it
    assert np.array_equal(cent.cpu().numpy(), ref_c)
    asg = ann.ann_ivf_assign(Xd, cent)
    torch.cuda.synchronize()
    ref_a = oracle.ivf_assign(X, ref_c)
    assert np.array_equal(asg.cpu().numpy(), ref_a)
    off, ids = ann.ann_ivf_group(asg.cpu().numpy(), nlist)
    roff, rids = oracle.ivf_lists(ref_a, nlist)
    assert np.array_equal(off, roff) and np.array_equal(ids, rids)


def test_empty_clusters_are_reseeded_like_the_oracle():
    # 300 points with only 40 distinct values and 64 centroids: clusters
    # empty out and are re-seeded by error order
    rng = np.random.default_rng(2)
    base = rng.standard_normal((40, 16)).astype(np.float32)
    X = base[rng.integers(0, 40, 300)]
    sample = np.arange(300, dtype=np.int64)
    init = rng.permutation(300)[:64].astype(np.int64)
    ref_c, ref_it, _ = oracle.ivf_train(X, 64, sample, init, max_iter=8)
    cent, it = ann.ann_ivf_train(dev(X), dev(sample), dev(init), 64, max_iter=8)
    torch.cuda.synchronize()
    say("reseed case: iterations", it, ref_it)
    assert it == ref_it and np.array_equal(cent.cpu().numpy(), ref_c)


def test_ties_take_the_lower_centroid():
    # duplicated centroids: every row is equidistant from both copies
    rng = np.random.default_rng(3)
    C = rng.standard_normal((8, 32)).astype(np.float32)
    C2 = np.repeat(C, 2, axis=0)
    X = (C[rng.integers(0, 8, 700)] + 0.1 * rng.standard_normal((700, 32))).astype(np.float32)
    asg = ann.ann_ivf_assign(dev(X), dev(C2)).cpu().numpy()
    assert np.array_equal(asg, oracle.ivf_assign(X, C2)) and np.all(asg % 2 == 0)


def test_bad_arguments():
    X = dev(np.zeros((100, 8), np.float32))
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_train(X, dev(np.arange(10, dtype=np.int64)), dev(np.arange(20, dtype=np.int64)), 20)
    assert e.value.code == ann.ANN_EINVAL   # sample smaller than nlist
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_train(X, dev(np.array([0, 5, 100], np.int64)), dev(np.arange(3, dtype=np.int64)), 3)
    assert e.value.code == ann.ANN_EINVAL   # sample id outside the rows
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_train(X, dev(np.arange(10, dtype=np.int64)), dev(np.array([0, 1, 10], np.int64)), 3)
    assert e.value.code == ann.ANN_EINVAL   # init outside the sample
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_group(np.array([0, 3, 1], np.int32), 3)
    assert e.value.code == ann.ANN_EINVAL


def test_empty_cluster_reseed_worked_example():
    """The hand-worked re-seed case of the CPU pins on 2-d rows (second
    coordinate 0): after one iteration 5, 30, -10; after two 2.5, 30, -10."""
    x = np.array([0.0, 0.0, 0.0, -10.0, 10.0, 30.0], np.float32)
    X = np.stack([x, np.zeros(6, np.float32)], axis=1)
    for iters, want in {1: [5.0, 30.0, -10.0], 2: [2.5, 30.0, -10.0]}.items():
        cent, it = ann.ann_ivf_train(dev(X), dev(np.arange(6, dtype=np.int64)),
                                     dev(np.array([0, 1, 2], np.int64)), 3, max_iter=iters)
        torch.cuda.synchronize()
        assert it == iters
        c = cent.cpu().numpy()
        assert c[:, 0].tolist() == want and not c[:, 1].any()
