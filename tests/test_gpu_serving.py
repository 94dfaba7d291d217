"""Continuous-batching server: every result equals the same query searched
alone (bit for bit: the arithmetic does not depend on the batch), under
Poisson arrivals with mixed k and ef, and under tight admission limits."""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1(gmm10k):
    X, g = gmm10k["X"], gmm10k["graph"]
    ix = ann.ann_index_create(g, "l2", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X))
    yield dict(ix=ix, X=X, Q=gmm10k["Q"], g=g)
    ix.close()


def alone(ix, q, k, ef, mode, rerank):
    r = ann.ann_search_ex(ix, mode, queries=torch.from_numpy(q[None]).to("cuda:0"), k=k, ef=ef,
                          rerank=rerank)
    torch.cuda.synchronize()
    return r["ids"][0].cpu().numpy(), r["dists"][0].cpu().numpy()


def drive(srv, Q, t_arr, qidx, ks, efs, timeout=60.0):
    got = {}
    t0 = time.perf_counter()
    i = 0
    while len(got) < len(t_arr):
        now = time.perf_counter() - t0
        assert now < timeout, "server did not finish in time"
        while i < len(t_arr) and t_arr[i] <= now:
            if not srv.submit(i, Q[qidx[i]], int(ks[i]), int(efs[i])):
                break
            i += 1
        for c in srv.poll():
            got[c["tag"]] = c
        time.sleep(1e-4)
    return got


@pytest.mark.parametrize("streams,max_inflight,max_batch", [(2, 4096, 512), (3, 3, 2), (1, 64, 64)])
def test_results_equal_alone(c1, streams, max_inflight, max_batch):
    mode, rerank = "f16", 20
    Q = c1["Q"]
    n = 300
    t_arr, qidx, ks, efs = synth.arrivals(1, n, 4000.0, n_pool=Q.shape[0])
    srv = ann.Server(c1["ix"], mode=mode, rerank=rerank, max_inflight=max_inflight,
                     max_batch=max_batch, streams=streams, k_max=100, ef_max=512)
    try:
        got = drive(srv, Q, t_arr, qidx, ks, efs)
    finally:
        srv.close()
    assert len(got) == n
    cache = {}
    for tag, c in got.items():
        assert c["status"] == 0
        key = (int(qidx[tag]), int(ks[tag]), int(efs[tag]))
        if key not in cache:
            cache[key] = alone(c1["ix"], Q[key[0]], key[1], key[2], mode, rerank)
        ids, d = cache[key]
        assert np.array_equal(c["ids"], ids[:key[1]]), tag
        assert np.array_equal(c["dists"], d[:key[1]]), tag
        assert c["t_submit"] <= c["t_start"] <= c["t_done"]


def test_matches_oracle_and_batches_overlap(c1):
    Q, X, g = c1["Q"], c1["X"], c1["g"]
    n = 400
    t_arr, qidx, ks, efs = synth.arrivals(2, n, 20000.0, k_choices=(10,), ef_choices=(128,),
                                          n_pool=Q.shape[0])
    srv = ann.Server(c1["ix"], mode="f32", rerank=0, max_inflight=4096, max_batch=64, streams=4,
                     k_max=10, ef_max=128)
    try:
        got = drive(srv, Q, t_arr, qidx, ks, efs)
    finally:
        srv.close()
    ref = oracle.hnsw_search(g, oracle.dense_store(X, "l2"), 10, 128, Q=Q)
    for tag, c in got.items():
        assert np.array_equal(c["ids"], ref["ids"][qidx[tag]])
        assert np.array_equal(c["dists"], ref["keys"][qidx[tag]])
    # several launches were on the device at the same time at least once
    spans = sorted({(c["t_start"], c["t_done"]) for c in got.values()})
    overlap = any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    print("batches:", len(spans), "overlapping:", overlap)
    assert len(spans) > 1


def test_queue_full_and_bad_requests(c1):
    srv = ann.Server(c1["ix"], mode="f32", max_inflight=1, max_batch=1, streams=1, k_max=10,
                     ef_max=64, queue_cap=2)
    try:
        q = c1["Q"][0]
        with pytest.raises(ann.AnnError) as e:
            srv.submit(0, q, 11, 10)          # k above k_max
        assert e.value.code == ann.ANN_EINVAL
        accepted = sum(srv.submit(i, q, 10, 64) for i in range(50))
        assert 1 <= accepted < 50             # the queue pushes back
        t0 = time.time()
        seen = 0
        while seen < accepted and time.time() - t0 < 30:
            seen += len(srv.poll())
            time.sleep(1e-3)
        assert seen == accepted
    finally:
        srv.close()
