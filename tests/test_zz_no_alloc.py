"""The brute-force entry point that allocates nothing (its scratch is a fixed
device array): through the C-ABI, two calls in a row (the second smaller)
equal ann_bruteforce bit for bit; a batch whose scratch would not fit is
refused on the host."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def call(fn_name, ix, Q, k):
    nq = Q.shape[0]
    q = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    ids = torch.full((nq, k), -7, dtype=torch.int64, device=DEV)
    dists = torch.full((nq, k), -7.0, dtype=torch.float32, device=DEV)
    cert = torch.full((nq,), -7, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    rc = getattr(ann.lib(), fn_name)(ix.handle, q.data_ptr(), nq, k, ids.data_ptr(),
                                     dists.data_ptr(), cert.data_ptr(), None)
    assert rc == ann.ANN_OK, ann.lib().ann_last_error().decode()
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dists.cpu().numpy(), cert.cpu().numpy()


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_noalloc_equals_bruteforce_on_two_calls(gmm10k, metric):
    X = gmm10k["X"].copy()
    g = gmm10k["graph"]
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    Qa = synth.gaussian_mixture(41, 700, 128, 16, 0.3, which="queries")
    Qb = Qa[:37] * 0.5
    ix = ann.ann_index_create(g, metric, 128, x_f32=X)
    try:
        for Q, k in ((Qa, 10), (Qb, 3)):          # the second call is smaller
            say(f"{metric}: {Q.shape[0]} queries, k={k}")
            a = call("ann_bruteforce_noalloc", ix, Q, k)
            b = call("ann_bruteforce", ix, Q, k)
            # ids and keys bit for bit; ann_bruteforce may certify by its
            # FP16 pass (2), the variant without allocation by FP32 tiles (1)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            assert np.all(a[2] == 1) and np.all(b[2] != 0)
    finally:
        ix.close()
    # and the oracle's exact scan agrees
    ref_ids, ref_k = oracle.bruteforce(oracle.dense_store(X, metric), X.shape[0], 3, Q=Qb,
                                       kmode="canon")
    assert np.array_equal(a[0], ref_ids) and np.array_equal(a[1], ref_k)


def test_noalloc_refuses_a_batch_beyond_its_scratch(gmm10k):
    X, g = gmm10k["X"], gmm10k["graph"]
    ix = ann.ann_index_create(g, "l2", 128, x_f32=X)
    try:
        # 512 bytes per query and row range: 2^16 queries cannot fit 32 MiB
        nq = 1 << 17
        q = torch.zeros((nq, 128), device=DEV)
        out = torch.empty((nq, 10), dtype=torch.int64, device=DEV)
        d = torch.empty((nq, 10), dtype=torch.float32, device=DEV)
        rc = ann.lib().ann_bruteforce_noalloc(ix.handle, q.data_ptr(), nq, 10, out.data_ptr(),
                                              d.data_ptr(), None, None)
        assert rc == ann.ANN_EBUDGET
        assert "split the batch" in ann.lib().ann_last_error().decode()
    finally:
        ix.close()
