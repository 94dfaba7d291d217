"""Brute force on matrix cores against the oracle's exact scan."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu


def check(X, Q, metric, k, g):
    ix = ann.ann_index_create(g, metric, X.shape[1], x_f32=X)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q).to("cuda:0"), k)
        torch.cuda.synchronize()
        ids, d, cert = ids.cpu().numpy(), d.cpu().numpy(), cert.cpu().numpy()
    finally:
        ix.close()
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X, metric), X.shape[0], k, Q=Q,
                                       kmode="canon")
    assert cert.all()
    assert np.array_equal(ids, ref_ids)
    assert np.array_equal(d, ref_k)


@pytest.mark.parametrize("k", [1, 10, 48])
def test_bruteforce_l2(gmm10k, k):
    print("bruteforce l2 k", k, flush=True)
    check(gmm10k["X"], gmm10k["Q"], "l2", k, gmm10k["graph"])


def test_bruteforce_ip_768(vmf_small):
    print("bruteforce ip 768", flush=True)
    check(vmf_small["X"], vmf_small["Q"], "ip", 10, vmf_small["graph"])


def test_half_pass_and_fp32_redo():
    """The FP16 preselection certifies what its wider bound allows (flag 2);
    the rest is redone by the FP32 tiles (flag 1).  Rows and queries near
    (1, ..., 1) have keys within a few hundredths of each other: the FP16
    bound (about 2^-10 of |q| |x| = 64) cannot separate them and the FP32
    one (about 1e-3) can, so nearly every query goes through the redo; on
    the Gaussian mixture the FP16 pass certifies them itself."""
    rng = np.random.default_rng(11)
    X = (1.0 + 0.01 * rng.standard_normal((3000, 64))).astype(np.float32)
    Q = (1.0 + 0.01 * rng.standard_normal((200, 64))).astype(np.float32)
    g = oracle.hnsw_build(X, "ip", 8, 32, np.zeros(X.shape[0]))
    ix = ann.ann_index_create(g, "ip", 64, x_f32=X)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q).to("cuda:0"), 10)
        torch.cuda.synchronize()
        ids, d, cert = ids.cpu().numpy(), d.cpu().numpy(), cert.cpu().numpy()
    finally:
        ix.close()
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X, "ip"), X.shape[0], 10, Q=Q,
                                       kmode="canon")
    assert np.array_equal(ids, ref_ids) and np.array_equal(d, ref_k)
    assert np.all(cert != 0) and np.mean(cert == 1) > 0.9, np.bincount(cert)


def test_values_beyond_the_fp16_range_take_the_fp32_tiles():
    """A query with a value beyond the FP16 range is saturated in the FP16
    pass, which then never certifies it: the FP32 tiles redo it (flag 1).
    Rows with such values switch the FP16 pass off for the whole index."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((2000, 32)).astype(np.float32)
    Q = rng.standard_normal((20, 32)).astype(np.float32)
    Q[3, 7] = 1.0e5                        # beyond 65504
    Q[11, 0] = -7.0e4
    g = oracle.hnsw_build(X, "ip", 8, 32, np.zeros(X.shape[0]))
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X, "ip"), X.shape[0], 10, Q=Q, kmode="canon")
    ix = ann.ann_index_create(g, "ip", 32, x_f32=X)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q).to("cuda:0"), 10)
        torch.cuda.synchronize()
        ids, d, cert = ids.cpu().numpy(), d.cpu().numpy(), cert.cpu().numpy()
    finally:
        ix.close()
    assert np.array_equal(ids, ref_ids) and np.array_equal(d, ref_k)
    assert cert[3] == 1 and cert[11] == 1 and np.all(cert != 0)
    # rows beyond the FP16 range (all scaled, so that the FP32 bound, which
    # grows with the largest value, still separates the keys): FP32 tiles only
    X2 = X * np.float32(1.0e5)
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X2, "ip"), X2.shape[0], 10, Q=Q, kmode="canon")
    ix = ann.ann_index_create(g, "ip", 32, x_f32=X2)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q).to("cuda:0"), 10)
        torch.cuda.synchronize()
        ids, d, cert = ids.cpu().numpy(), d.cpu().numpy(), cert.cpu().numpy()
    finally:
        ix.close()
    assert np.array_equal(ids, ref_ids) and np.array_equal(d, ref_k)
    assert np.all(cert == 1)


def test_half_pass_certifies_the_mixture(gmm10k):
    X, Q, g = gmm10k["X"], gmm10k["Q"], gmm10k["graph"]
    ix = ann.ann_index_create(g, "l2", X.shape[1], x_f32=X)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q).to("cuda:0"), 10)
        torch.cuda.synchronize()
        cert = cert.cpu().numpy()
    finally:
        ix.close()
    assert np.all(cert != 0) and np.mean(cert == 2) > 0.9, np.bincount(cert)


def test_bruteforce_ragged_and_tiny():
    # n not a multiple of the 128-row tile, nq not a multiple of 128, n < k
    rng = np.random.default_rng(3)
    X = rng.standard_normal((1000 + 37, 64)).astype(np.float32)
    Q = rng.standard_normal((131, 64)).astype(np.float32)
    g = oracle.hnsw_build(X, "ip", 8, 32, np.zeros(X.shape[0]))
    check(X, Q, "ip", 10, g)
    # d not a multiple of the 32-dimension stage (the last stage is half empty)
    X48 = rng.standard_normal((777, 48)).astype(np.float32)
    Q48 = rng.standard_normal((300, 48)).astype(np.float32)
    g48 = oracle.hnsw_build(X48, "l2", 8, 32, np.zeros(X48.shape[0]))
    check(X48, Q48, "l2", 16, g48)
    Xs = X[:5]
    gs = oracle.hnsw_build(Xs, "l2", 4, 8, np.zeros(5))
    ix = ann.ann_index_create(gs, "l2", 64, x_f32=Xs)
    try:
        ids, d, cert = ann.ann_bruteforce(ix, torch.from_numpy(Q[:3]).to("cuda:0"), 8)
        ids = ids.cpu().numpy()
        assert np.all(ids[:, 5:] == -1) and np.all(np.sort(ids[:, :5], 1) == np.arange(5))
    finally:
        ix.close()


def test_bruteforce_rejects_bad_k(gmm10k):
    ix = ann.ann_index_create(gmm10k["graph"], "l2", 128, x_f32=gmm10k["X"])
    try:
        with pytest.raises(ann.AnnError):
            ann.ann_bruteforce(ix, torch.zeros((2, 128), device="cuda:0"), 49)
    finally:
        ix.close()


def test_calls_on_two_streams_share_the_scratch_safely(gmm10k):
    """Back-to-back asynchronous calls on two streams use the index's one
    candidate buffer in turn: each result equals the oracle's exact scan."""
    X, Q = gmm10k["X"], gmm10k["Q"]
    ix = ann.ann_index_create(gmm10k["graph"], "l2", 128, x_f32=X)
    try:
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        q1 = torch.from_numpy(Q[:64]).to("cuda:0")
        q2 = torch.from_numpy(Q[64:]).to("cuda:0")
        torch.cuda.synchronize()
        outs = []
        for rep in range(3):
            outs.append(ann.ann_bruteforce(ix, q1, 10, stream=s1))
            outs.append(ann.ann_bruteforce(ix, q2, 10, stream=s2))
        torch.cuda.synchronize()
    finally:
        ix.close()
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X, "l2"), X.shape[0], 10, Q=Q,
                                       kmode="canon")
    for j, (ids, d, cert) in enumerate(outs):
        sl = slice(0, 64) if j % 2 == 0 else slice(64, None)
        assert cert.cpu().numpy().all()
        assert np.array_equal(ids.cpu().numpy(), ref_ids[sl]), j
        assert np.array_equal(d.cpu().numpy(), ref_k[sl]), j
