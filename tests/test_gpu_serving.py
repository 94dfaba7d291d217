"""Serving with per-slot admission: every served result equals the same
query searched alone (bit for bit: the arithmetic does not depend on what
else runs), under Poisson arrivals with mixed k and ef and under tight
admission limits; requests that arrive while others run start on a free
slot and overlap them on the device (shown with the kernel's own clock)."""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-serving]", *a, flush=True)


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


def wait_all(srv, n, timeout=60.0):
    got = {}
    t0 = time.perf_counter()
    while len(got) < n:
        assert time.perf_counter() - t0 < timeout, "server did not finish in time"
        for c in srv.poll():
            got[c["tag"]] = c
        time.sleep(1e-4)
    return got


@pytest.mark.parametrize("max_inflight,slots", [(4096, 0), (3, 2), (64, 1), (7, 0)])
def test_results_equal_alone(c1, max_inflight, slots):
    mode, rerank = "f16", 20
    Q = c1["Q"]
    n = 300
    t_arr, qidx, ks, efs = synth.arrivals(1, n, 4000.0, n_pool=Q.shape[0])
    say(f"poisson 4000/s, ring {max_inflight}, slots {slots}")
    srv = ann.Server(c1["ix"], mode=mode, rerank=rerank, max_inflight=max_inflight, slots=slots,
                     k_max=100, ef_max=512)
    try:
        st = srv.info()
        assert st["ring"] == max_inflight and st["slots"] >= 1
        if slots:
            assert st["slots"] == slots
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
        assert c["d_start"] <= c["d_done"]
        assert 0 <= c["slot"] < st["slots"]


def test_matches_oracle_and_requests_overlap_on_the_device(c1):
    Q, X, g = c1["Q"], c1["X"], c1["g"]
    n = 400
    t_arr, qidx, ks, efs = synth.arrivals(2, n, 20000.0, k_choices=(10,), ef_choices=(128,),
                                          n_pool=Q.shape[0])
    srv = ann.Server(c1["ix"], mode="f32", rerank=0, max_inflight=4096, k_max=10, ef_max=128)
    try:
        got = drive(srv, Q, t_arr, qidx, ks, efs)
        nslots = srv.info()["slots"]
    finally:
        srv.close()
    ref = oracle.hnsw_search(g, oracle.dense_store(X, "l2"), 10, 128, Q=Q)
    for tag, c in got.items():
        assert np.array_equal(c["ids"], ref["ids"][qidx[tag]])
        assert np.array_equal(c["dists"], ref["keys"][qidx[tag]])
    # device intervals of requests submitted at different times intersect:
    # a request started while an earlier one was still running
    iv = sorted((c["d_start"], c["d_done"], c["t_submit"], c["slot"]) for c in got.values())
    pairs = sum(1 for a, b in zip(iv, iv[1:]) if b[0] < a[1] and b[2] != a[2] and b[3] != a[3])
    say(f"{len(iv)} requests on {nslots} slots, {pairs} consecutive overlapping pairs, "
        f"{len({c['slot'] for c in got.values()})} slots used")
    assert pairs > 0


def test_a_freed_slot_takes_the_next_request_at_once(c1):
    """Four slots busy with beams of very different widths; short requests
    submitted behind them start as soon as the narrowest beam frees its slot
    and finish while the widest is still running (a batch-granular server
    would hold them until all four were done)."""
    Q, X, g = c1["Q"], c1["X"], c1["g"]
    srv = ann.Server(c1["ix"], mode="f32", rerank=0, max_inflight=64, slots=4, k_max=10,
                     ef_max=8000)
    long_efs = [100, 1000, 3000, 8000]
    try:
        for i, ef in enumerate(long_efs):
            assert srv.submit(i, Q[i], 10, ef)
        time.sleep(5e-4)
        for j in range(8):
            assert srv.submit(100 + j, Q[10 + j], 10, 16)
        got = wait_all(srv, len(long_efs) + 8)
    finally:
        srv.close()
    longs = [got[i] for i in range(len(long_efs))]
    shorts = [got[100 + j] for j in range(8)]
    widest = longs[-1]
    say("long beams (device ms):", [round((c["d_done"] - c["d_start"]) * 1e3, 3) for c in longs])
    say("short requests start/finish vs the widest beam's end (device ms):",
        [(round((c["d_start"] - widest["d_done"]) * 1e3, 3),
          round((c["d_done"] - widest["d_done"]) * 1e3, 3)) for c in shorts])
    # the four long requests were claimed first, so every short one waited for
    # a slot to free, and all of them were done before the widest beam
    assert all(c["d_start"] >= min(l["d_done"] for l in longs) for c in shorts)
    assert all(c["d_done"] < widest["d_done"] for c in shorts)
    # every result is still the oracle's
    st = oracle.dense_store(X, "l2")
    for i, ef in enumerate(long_efs):
        r = oracle.hnsw_search(g, st, 10, ef, Q=Q[i:i + 1])
        assert np.array_equal(longs[i]["ids"], r["ids"][0])
    r = oracle.hnsw_search(g, st, 10, 16, Q=Q[10:18])
    for j in range(8):
        assert np.array_equal(shorts[j]["ids"], r["ids"][j])


def test_kernel_relaunches_after_idle(c1):
    Q = c1["Q"]
    srv = ann.Server(c1["ix"], mode="f32", max_inflight=16, k_max=10, ef_max=64, idle_us=200)
    try:
        outs = []
        for rnd in range(3):
            assert srv.submit(rnd, Q[rnd], 10, 64)
            outs.append(wait_all(srv, 1)[rnd])
            time.sleep(0.02)          # far beyond idle_us: the kernel has ended
        for rnd, c in enumerate(outs):
            ids, d = alone(c1["ix"], Q[rnd], 10, 64, "f32", 0)
            assert np.array_equal(c["ids"], ids) and np.array_equal(c["dists"], d)
    finally:
        srv.close()


def test_destroy_with_requests_in_flight_returns(c1):
    Q = c1["Q"]
    srv = ann.Server(c1["ix"], mode="f32", max_inflight=32, slots=2, k_max=10, ef_max=4000)
    for i in range(64):
        srv.submit(i, Q[i % Q.shape[0]], 10, 4000)
    t0 = time.perf_counter()
    srv.close()
    say(f"destroy with 64 wide requests queued: {time.perf_counter() - t0:.3f}s")
    assert time.perf_counter() - t0 < 30


def test_queue_full_and_bad_requests(c1):
    srv = ann.Server(c1["ix"], mode="f32", max_inflight=1, slots=1, k_max=10, ef_max=64,
                     queue_cap=2)
    try:
        q = c1["Q"][0]
        with pytest.raises(ann.AnnError) as e:
            srv.submit(0, q, 11, 10)          # k above k_max
        assert e.value.code == ann.ANN_EINVAL
        with pytest.raises(ann.AnnError) as e:
            srv.submit(0, q, 10, 65)          # ef above ef_max
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


def test_bad_configurations(c1):
    with pytest.raises(ann.AnnError) as e:
        ann.Server(c1["ix"], mode="pq", k_max=10, ef_max=64)
    assert e.value.code in (ann.ANN_EINVAL, ann.ANN_EUNSUP)
    with pytest.raises(ann.AnnError) as e:
        ann.Server(c1["ix"], mode="f32", max_inflight=0, k_max=10, ef_max=64)
    assert e.value.code == ann.ANN_EINVAL
    with pytest.raises(ann.AnnError) as e:
        ann.Server(c1["ix"], mode="f32", k_max=10, ef_max=64, hbm_budget=1)
    assert e.value.code == ann.ANN_EBUDGET
