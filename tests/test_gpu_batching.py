"""Batching: the autotuner and captured (HIP graph) batches.

The autotuner only changes the launch shape, never the arithmetic, so
results after tuning still equal the oracle's bit for bit.  A plan replays
one captured launch with its batch size read from device memory: every
replay, with other work and synchronizations between replays and on
different streams, equals the oracle's search of the queries in its buffer.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-batching]", *a, flush=True)


@pytest.fixture(scope="module")
def c1(gmm10k):
    X, g = gmm10k["X"], gmm10k["graph"]
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=4)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(g, "l2", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X),
                              pq_codebook=cb, pq_codes=codes)
    yield dict(ix=ix, X=X, Q=gmm10k["Q"], g=g, cb=cb, codes=codes)
    ix.close()


def store(c, mode):
    if mode == "f32":
        return oracle.dense_store(c["X"], "l2")
    if mode == "f16":
        return oracle.dense_store(oracle.to_f16(c["X"]), "l2", "f16")
    return oracle.pq_store(c["cb"], c["codes"], "l2")


def same(ids, dists, ref, rows=slice(None)):
    assert np.array_equal(ids, ref["ids"][rows])
    assert np.array_equal(dists, ref["keys"][rows])


@pytest.mark.parametrize("mode,rerank", [("f32", 0), ("f16", 20), ("pq", 30)])
def test_autotune_picks_a_valid_shape_and_keeps_results(c1, mode, rerank):
    ix, Q = c1["ix"], c1["Q"]
    q = torch.from_numpy(np.ascontiguousarray(np.tile(Q, (4, 1)))).to(DEV)
    say("autotune", mode)
    best = ann.ann_autotune(ix, mode, queries=q, k=10, ef=96, rerank=rerank)
    say("chosen", best)
    assert best["waves_per_query"] in (1, 2, 4, 8)
    assert best["lanes_per_row"] in (16, 32, 64)
    assert best["slots"] >= 0
    assert ann.ann_get_launch(ix, mode) == best
    r = ann.ann_search_ex(ix, mode, queries=q[:Q.shape[0]], k=10, ef=96, rerank=rerank)
    torch.cuda.synchronize()
    ref = oracle.hnsw_search(c1["g"], store(c1, mode), 10, 96, Q=Q,
                             rerank_f32=c1["X"] if rerank else None, rerank=rerank)
    same(r["ids"].cpu().numpy(), r["dists"].cpu().numpy(), ref)
    ann.ann_set_launch(ix, mode)     # back to the defaults for the other tests


def test_plan_replays_equal_the_oracle(c1):
    ix, Q = c1["ix"], c1["Q"]
    nq_all = Q.shape[0]
    ref = oracle.hnsw_search(c1["g"], store(c1, "f16"), 10, 64, Q=Q, rerank_f32=c1["X"],
                             rerank=20)
    plan = ann.Plan(ix, "f16", capacity=nq_all, k=10, ef=64, rerank=20)
    try:
        info = plan.info()
        say("plan launch shape", info)
        assert info["slots"] >= 1
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        order = np.arange(nq_all)
        # replays with different contents and sizes; eager work in between
        for rep, (nq, stream) in enumerate([(nq_all, None), (37, s1), (nq_all, s2), (1, s1),
                                            (64, None)]):
            order = np.roll(order, 17)
            plan.queries[:nq].copy_(torch.from_numpy(Q[order[:nq]]).to(DEV))
            torch.cuda.synchronize()
            plan.launch(nq, stream=stream)
            # unrelated eager work on the default stream while the replay runs
            x = torch.randn((512, 512), device=DEV)
            (x @ x).sum().item()
            direct = ann.ann_search_ex(ix, "f16", queries=torch.from_numpy(Q[:8]).to(DEV), k=10,
                                       ef=64, rerank=20)
            torch.cuda.synchronize()
            same(direct["ids"].cpu().numpy(), direct["dists"].cpu().numpy(), ref, slice(0, 8))
            say(f"replay {rep}: nq={nq}")
            same(plan.ids[:nq].cpu().numpy(), plan.dists[:nq].cpu().numpy(), ref, order[:nq])
            assert np.all(plan.status[:nq].cpu().numpy() == 0)
    finally:
        plan.close()


def test_plan_with_per_query_k_and_ef(c1):
    ix, Q = c1["ix"], c1["Q"]
    rng = np.random.default_rng(4)
    ks = rng.choice([1, 5, 10, 20], size=Q.shape[0]).astype(np.int32)
    efs = rng.choice([8, 32, 100], size=Q.shape[0]).astype(np.int32)
    plan = ann.Plan(ix, "f32", capacity=Q.shape[0], k=10, ef=64, k_max=20, ef_max=100,
                    per_query=True)
    try:
        for rep in range(3):
            plan.queries.copy_(torch.from_numpy(Q).to(DEV))
            plan.k.copy_(torch.from_numpy(ks).to(DEV))
            plan.ef.copy_(torch.from_numpy(efs).to(DEV))
            torch.cuda.synchronize()
            plan.launch(Q.shape[0])
            torch.cuda.synchronize()
            ids = plan.ids.cpu().numpy()
            for i in range(Q.shape[0]):
                r = oracle.hnsw_search(c1["g"], store(c1, "f32"), int(ks[i]), int(efs[i]),
                                       Q=Q[i:i + 1])
                assert np.array_equal(ids[i, :ks[i]], r["ids"][0]), (rep, i)
                assert np.all(ids[i, ks[i]:] == -1)
            ks, efs = ks[::-1].copy(), efs[::-1].copy()
    finally:
        plan.close()


def test_plan_rejects_bad_arguments(c1):
    with pytest.raises(ann.AnnError) as e:
        ann.Plan(c1["ix"], "f32", capacity=10, k=10, ef=ann.ANN_EF_MAX + 1)
    assert e.value.code == ann.ANN_EBUDGET
