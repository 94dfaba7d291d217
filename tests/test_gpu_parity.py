"""GPU parity: the HIP search against the CPU oracle on the same seeded inputs.

Every key is evaluated in the same fixed FP32 order on both sides, so ids,
keys, visited sets and expansion counts must agree exactly.
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
    print("[gpu-parity]", *a, flush=True)


@pytest.fixture(scope="module")
def c1(gmm10k):
    X, g = gmm10k["X"], gmm10k["graph"]
    f8, s8 = oracle.encode_fp8_rows(X)
    ix = ann.ann_index_create(g, "l2", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X),
                              x_bf16=oracle.to_bf16(X), x_fp8=f8, fp8_scale=s8)
    yield dict(ix=ix, X=X, Q=gmm10k["Q"], g=g, f8=f8, s8=s8)
    ix.close()


@pytest.fixture(scope="module")
def v768(vmf_small):
    X, g = vmf_small["X"], vmf_small["graph"]
    f8, s8 = oracle.encode_fp8_rows(X)
    ix = ann.ann_index_create(g, "ip", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X),
                              x_bf16=oracle.to_bf16(X), x_fp8=f8, fp8_scale=s8)
    yield dict(ix=ix, X=X, Q=vmf_small["Q"], g=g, f8=f8, s8=s8)
    ix.close()


def store_for(data, mode, metric):
    X = data["X"]
    if mode == "f32":
        return oracle.dense_store(X, metric)
    if mode == "f16":
        return oracle.dense_store(oracle.to_f16(X), metric, "f16")
    if mode == "bf16":
        return oracle.dense_store(oracle.to_bf16(X), metric, "bf16")
    return oracle.dense_store(data["f8"], metric, "fp8", fp8_scale=data["s8"])


def gpu(ix, mode, Q, k, ef, rerank=0, visited_cap=0, k_max=None, ef_max=None):
    q = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    kk = torch.from_numpy(np.asarray(k, np.int32)).to(DEV) if np.ndim(k) else k
    ee = torch.from_numpy(np.asarray(ef, np.int32)).to(DEV) if np.ndim(ef) else ef
    r = ann.ann_search_ex(ix, mode, queries=q, k=kk, ef=ee, rerank=rerank, want_stats=True,
                          visited_cap=visited_cap, k_max=k_max, ef_max=ef_max)
    torch.cuda.synchronize()
    return {k_: v.cpu().numpy() for k_, v in r.items()}


def assert_same(got, ref, visited=False):
    assert np.array_equal(got["ids"], ref["ids"]), np.argwhere(got["ids"] != ref["ids"])[:5]
    assert np.array_equal(got["dists"], ref["keys"])
    assert np.array_equal(got["stats"][:, 1], ref["stats"][:, 2])   # layer-0 expansions
    assert np.array_equal(got["stats"][:, 2], ref["stats"][:, 3])   # |visited|
    assert np.array_equal(got["stats"][:, 3], ref["stats"][:, 4])   # |W|
    assert np.all(got["status"] == 0)
    if visited:
        for a, b in zip(got["visited"], ref["visited"]):
            assert np.array_equal(np.sort(a[a >= 0]), b[b >= 0])


@pytest.mark.parametrize("ef", [1, 10, 64, 200, 700])
def test_f32_l2_bitexact(c1, ef):
    say("f32 l2 gmm10k ef", ef)
    ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), 10, ef, Q=c1["Q"],
                             visited_cap=4096)
    got = gpu(c1["ix"], "f32", c1["Q"], 10, ef, visited_cap=4096)
    assert_same(got, ref, visited=True)


@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("slots", [1, 7, 0])
def test_launch_shape_does_not_change_results(c1, lanes, slots):
    say("launch shape", lanes, slots)
    ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), 10, 64, Q=c1["Q"])
    ann.ann_set_launch(c1["ix"], "f32", slots=slots, lanes_per_row=lanes)
    try:
        got = gpu(c1["ix"], "f32", c1["Q"], 10, 64)
    finally:
        ann.ann_set_launch(c1["ix"], "f32", 0, 0)
    assert_same(got, ref)


@pytest.mark.parametrize("mode", ["f16", "bf16", "fp8"])
@pytest.mark.parametrize("rerank", [0, 40])
def test_reduced_precision_l2_bitexact(c1, mode, rerank):
    say("reduced precision l2", mode, rerank)
    st = store_for(c1, mode, "l2")
    ref = oracle.hnsw_search(c1["g"], st, 10, 64, Q=c1["Q"], rerank_f32=c1["X"] if rerank else None,
                             rerank=rerank)
    got = gpu(c1["ix"], mode, c1["Q"], 10, 64, rerank=rerank)
    assert_same(got, ref)


@pytest.mark.parametrize("mode", ["f32", "f16", "bf16", "fp8"])
@pytest.mark.parametrize("lanes", [32, 64])
def test_768d_ip_bitexact(v768, mode, lanes):
    say("768-d ip", mode, lanes)
    st = store_for(v768, mode, "ip")
    rr = 0 if mode == "f32" else 40
    ref = oracle.hnsw_search(v768["g"], st, 10, 100, Q=v768["Q"],
                             rerank_f32=v768["X"] if rr else None, rerank=rr, visited_cap=4096)
    # 768-d rows: 192 FP32 chunks need 64 lanes; 96 16-bit chunks fit 32 lanes
    # (3 per lane), 48 FP8 chunks fit 32 lanes (2 per lane)
    shape_ok = lanes == 64 or mode != "f32"
    if not shape_ok:
        with pytest.raises(ann.AnnError):
            ann.ann_set_launch(v768["ix"], mode, lanes_per_row=lanes)
        return
    ann.ann_set_launch(v768["ix"], mode, lanes_per_row=lanes)
    try:
        got = gpu(v768["ix"], mode, v768["Q"], 10, 100, rerank=rr, visited_cap=4096)
    finally:
        ann.ann_set_launch(v768["ix"], mode, 0, 0)
    assert_same(got, ref, visited=True)


def test_mixed_k_ef_in_one_launch_equals_alone(c1):
    rng = np.random.default_rng(0)
    nq = c1["Q"].shape[0]
    k = rng.choice([1, 10, 100], nq).astype(np.int32)
    ef = rng.choice([16, 64, 128, 512], nq).astype(np.int32)
    say("mixed k/ef")
    got = gpu(c1["ix"], "f32", c1["Q"], k, ef, k_max=100, ef_max=512)
    ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), k, ef, Q=c1["Q"])
    assert_same(got, ref)
    for i in (0, 5, 17):
        alone = gpu(c1["ix"], "f32", c1["Q"][i:i + 1], int(k[i]), int(ef[i]))
        kk = int(k[i])
        assert np.array_equal(alone["ids"][0, :kk], got["ids"][i, :kk])
        assert np.array_equal(alone["dists"][0, :kk], got["dists"][i, :kk])
        assert np.all(got["ids"][i, kk:] == -1)


def test_pq_adc_bitexact(c1):
    X = c1["X"]
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=8)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(c1["g"], "l2", X.shape[1], x_f32=X, pq_codebook=cb, pq_codes=codes)
    try:
        for rr in (0, 50):
            say("pq adc rerank", rr)
            ref = oracle.hnsw_search(c1["g"], oracle.pq_store(cb, codes, "l2"), 10, 64, Q=c1["Q"],
                                     rerank_f32=X if rr else None, rerank=rr)
            got = gpu(ix, "pq", c1["Q"], 10, 64, rerank=rr)
            assert_same(got, ref)
    finally:
        ix.close()


@pytest.mark.parametrize("m", [64, 48, 16])
def test_pq_lane_groups_bitexact(v768, m):
    """PQ on the 4,096 x 768 IP set with m = 64, 48 and 16 subspaces, scored
    by 16, 32 and 64 lanes per candidate, with 1 and 2 waves per query (HNSW
    expansions take the lane-group schedule, long candidate runs one lane per
    row): ids, keys, visited counts and |W| equal the oracle's."""
    X = v768["X"]
    sample, init = synth.pq_sample(0, X.shape[0], X.shape[0], 256)
    cb, _, _ = oracle.pq_train(X, m, 256, sample, init, max_iter=3)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(v768["g"], "ip", X.shape[1], x_f32=X, pq_codebook=cb, pq_codes=codes)
    try:
        ref = oracle.hnsw_search(v768["g"], oracle.pq_store(cb, codes, "ip"), 10, 80, Q=v768["Q"],
                                 rerank_f32=X, rerank=40)
        for lanes in (16, 32, 64):
            for waves in (1, 2):
                say(f"pq m={m} lanes={lanes} waves={waves}")
                ann.ann_set_launch(ix, "pq", lanes_per_row=lanes, waves_per_query=waves)
                assert ann.ann_get_launch(ix, "pq")["lanes_per_row"] == lanes
                assert_same(gpu(ix, "pq", v768["Q"], 10, 80, rerank=40), ref)
    finally:
        ix.close()


def test_sparse_bitexact(sparse_small):
    s = sparse_small
    ix = ann.ann_index_create(s["graph"], "ip", s["vocab"], sp_indptr=s["indptr"], sp_ids=s["ids"],
                              sp_vals=s["vals"])
    try:
        qp, qi, qv = s["q"]
        sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
              torch.from_numpy(qv).to(DEV))
        for ef in (10, 100):
            say("sparse ef", ef)
            r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=ef, want_stats=True)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in r.items()}
            ref = oracle.hnsw_search(s["graph"], s["store"], 10, ef, sparse_q=s["q"])
            assert_same(got, ref)
    finally:
        ix.close()


def test_sparse_query_above_256_terms_is_truncated_and_flagged(sparse_small):
    """A sparse query keeps at most 256 terms on the device: longer ones are
    searched with their first 256 (by position) and flagged with status bit 2;
    exactly 256 terms is searched whole."""
    s = sparse_small
    rng = np.random.default_rng(21)
    lens = [256, 257, 300, 40]
    rows = [np.sort(rng.choice(s["vocab"], size=m, replace=False)).astype(np.uint16) for m in lens]
    vals = [rng.lognormal(0.0, 0.5, size=m).astype(np.float32) for m in lens]
    qp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    qi = np.concatenate(rows)
    qv = np.concatenate(vals)
    # what the device searches: each query cut to its first 256 terms
    cut = [min(m, 256) for m in lens]
    tp = np.concatenate([[0], np.cumsum(cut)]).astype(np.int64)
    ti = np.concatenate([r[:c] for r, c in zip(rows, cut)])
    tv = np.concatenate([v[:c] for v, c in zip(vals, cut)])
    ix = ann.ann_index_create(s["graph"], "ip", s["vocab"], sp_indptr=s["indptr"], sp_ids=s["ids"],
                              sp_vals=s["vals"])
    try:
        sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
              torch.from_numpy(qv).to(DEV))
        r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=64, want_stats=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in r.items()}
    finally:
        ix.close()
    assert got["status"].tolist() == [0, 2, 2, 0]
    ref = oracle.hnsw_search(s["graph"], s["store"], 10, 64, sparse_q=(tp, ti, tv))
    assert np.array_equal(got["ids"], ref["ids"])
    assert np.array_equal(got["dists"], ref["keys"])
    # the untruncated 300-term query ranks differently in the oracle
    full = oracle.hnsw_search(s["graph"], s["store"], 10, 64, sparse_q=(qp, qi, qv))
    assert not np.array_equal(full["keys"][2], ref["keys"][2])


@pytest.mark.parametrize("d,metric", [(1536, "l2"), (2048, "ip")])
def test_rerank_above_1024_dimensions(d, metric):
    """FP32 rerank of rows wider than 1,024 floats (more than one round of
    256 chunks per lane): FP16 traversal + rerank of 30 equals the oracle."""
    n, nq = 1200, 16
    X = synth.gaussian_mixture(31, n, d, 8, 0.3)
    Q = synth.gaussian_mixture(31, nq, d, 8, 0.3, which="queries")
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    g = oracle.hnsw_build(X, metric, 8, 32, synth.level_uniforms(31, n))
    say(f"rerank at d={d} {metric}")
    ix = ann.ann_index_create(g, metric, d, x_f32=X, x_f16=oracle.to_f16(X))
    try:
        got = gpu(ix, "f16", Q, 10, 40, rerank=30)
    finally:
        ix.close()
    ref = oracle.hnsw_search(g, oracle.dense_store(oracle.to_f16(X), metric, "f16"), 10, 40, Q=Q,
                             rerank_f32=X, rerank=30)
    assert_same(got, ref)


def test_edge_cases(c1):
    ix = c1["ix"]
    # nq = 0 is a no-op
    q0 = torch.zeros((0, 128), device=DEV)
    r = ann.ann_search_ex(ix, "f32", queries=q0, k=10, ef=10)
    assert r["ids"].shape == (0, 10)
    # ef < k behaves as ef = k
    a = gpu(ix, "f32", c1["Q"][:5], 20, 5)
    b = gpu(ix, "f32", c1["Q"][:5], 20, 20)
    assert np.array_equal(a["ids"], b["ids"])
    # over-capacity requests fail on the host
    with pytest.raises(ann.AnnError) as e:
        gpu(ix, "f32", c1["Q"][:2], 10, ann.ANN_EF_MAX + 1)
    assert e.value.code == ann.ANN_EBUDGET
    # a 3-node graph: fewer nodes than k -> padding
    X = np.zeros((3, 16), np.float32); X[:, 0] = [0, 1, 5]
    g = oracle.hnsw_build(X, "l2", 4, 8, np.zeros(3))
    tiny = ann.ann_index_create(g, "l2", 16, x_f32=X)
    try:
        got = gpu(tiny, "f32", X[:1], 5, 8)
        assert got["ids"][0].tolist() == [0, 1, 2, -1, -1]
        assert np.isinf(got["dists"][0, 3:]).all()
    finally:
        tiny.close()
    # a single node
    one = oracle.hnsw_build(X[:1], "l2", 4, 8, np.zeros(1))
    single = ann.ann_index_create(one, "l2", 16, x_f32=X[:1])
    try:
        got = gpu(single, "f32", X[1:3], 2, 4)
        assert got["ids"][:, 0].tolist() == [0, 0] and np.all(got["ids"][:, 1] == -1)
    finally:
        single.close()


def test_ann_search_blocking_api(c1):
    q = torch.from_numpy(c1["Q"]).to(DEV)
    ids, d = ann.ann_search(c1["ix"], q, 10, 64)
    ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), 10, 64, Q=c1["Q"])
    assert np.array_equal(ids.cpu().numpy(), ref["ids"])
    assert np.array_equal(d.cpu().numpy(), ref["keys"])


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_waves_per_query_do_not_change_results(c1, v768, sparse_small, waves):
    say("waves per query", waves)
    # dense L2, with and without rerank
    for mode, rr in (("f32", 0), ("f16", 40)):
        st = store_for(c1, mode, "l2")
        ref = oracle.hnsw_search(c1["g"], st, 10, 200, Q=c1["Q"], rerank_f32=c1["X"] if rr else None,
                                 rerank=rr, visited_cap=4096)
        ann.ann_set_launch(c1["ix"], mode, waves_per_query=waves)
        try:
            got = gpu(c1["ix"], mode, c1["Q"], 10, 200, rerank=rr, visited_cap=4096)
        finally:
            ann.ann_set_launch(c1["ix"], mode, 0, 0, 0)
        assert_same(got, ref, visited=True)
    # 768-d inner product
    ref = oracle.hnsw_search(v768["g"], store_for(v768, "bf16", "ip"), 10, 300, Q=v768["Q"],
                             rerank_f32=v768["X"], rerank=40)
    ann.ann_set_launch(v768["ix"], "bf16", waves_per_query=waves)
    try:
        got = gpu(v768["ix"], "bf16", v768["Q"], 10, 300, rerank=40)
    finally:
        ann.ann_set_launch(v768["ix"], "bf16", 0, 0, 0)
    assert_same(got, ref)
    # sparse
    s = sparse_small
    ix = ann.ann_index_create(s["graph"], "ip", s["vocab"], sp_indptr=s["indptr"], sp_ids=s["ids"],
                              sp_vals=s["vals"])
    try:
        qp, qi, qv = s["q"]
        sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
              torch.from_numpy(qv).to(DEV))
        ann.ann_set_launch(ix, "sparse", waves_per_query=waves)
        r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=100, want_stats=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in r.items()}
        assert_same(got, oracle.hnsw_search(s["graph"], s["store"], 10, 100, sparse_q=s["q"]))
    finally:
        ix.close()


def test_pq_with_waves(c1):
    X = c1["X"]
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=4)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(c1["g"], "l2", X.shape[1], x_f32=X, pq_codebook=cb, pq_codes=codes)
    try:
        ref = oracle.hnsw_search(c1["g"], oracle.pq_store(cb, codes, "l2"), 10, 100, Q=c1["Q"],
                                 rerank_f32=X, rerank=30)
        for waves in (2, 4, 8):
            say("pq waves", waves)
            ann.ann_set_launch(ix, "pq", waves_per_query=waves)
            assert_same(gpu(ix, "pq", c1["Q"], 10, 100, rerank=30), ref)
    finally:
        ix.close()


@pytest.mark.parametrize("buf,place", [(64, "lds"), (200, "lds"), (-1, "lds"), (0, "auto"),
                                       (64, "hbm"), (0, "hbm")])
def test_beam_layouts_do_not_change_results(c1, v768, sparse_small, buf, place):
    """The insert buffer of a wide beam, and a beam list kept in HBM, hold the
    same W as one sorted list in LDS: forced small buffers (many flushes,
    cuts from both tails) at every beam width, the automatic choice (buffer
    above ef 1024, HBM list above 4096), none, and the HBM list."""
    say("beam layout", buf, place)
    ann.ann_set_launch(c1["ix"], "f32", beam_buffer=buf, beam_list=place)
    try:
        for ef in (1, 10, 64, 700, 2000, 5000):
            ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), 10, ef, Q=c1["Q"],
                                     visited_cap=10000)
            assert_same(gpu(c1["ix"], "f32", c1["Q"], 10, ef, visited_cap=10000), ref, visited=True)
        rng = np.random.default_rng(1)
        nq = c1["Q"].shape[0]
        k = rng.choice([1, 10, 100], nq).astype(np.int32)
        ef = rng.choice([16, 100, 1500, 3000], nq).astype(np.int32)
        ref = oracle.hnsw_search(c1["g"], oracle.dense_store(c1["X"], "l2"), k, ef, Q=c1["Q"])
        assert_same(gpu(c1["ix"], "f32", c1["Q"], k, ef, k_max=100, ef_max=3000), ref)
    finally:
        ann.ann_set_launch(c1["ix"], "f32")
    # 768-d inner product, FP16 rows and FP32 rerank, several waves
    ann.ann_set_launch(v768["ix"], "f16", waves_per_query=4, beam_buffer=buf, beam_list=place)
    try:
        ref = oracle.hnsw_search(v768["g"], store_for(v768, "f16", "ip"), 10, 1200, Q=v768["Q"],
                                 rerank_f32=v768["X"], rerank=40)
        assert_same(gpu(v768["ix"], "f16", v768["Q"], 10, 1200, rerank=40), ref)
    finally:
        ann.ann_set_launch(v768["ix"], "f16")
    # sparse rows
    if buf > 0:
        s = sparse_small
        ix = ann.ann_index_create(s["graph"], "ip", s["vocab"], sp_indptr=s["indptr"],
                                  sp_ids=s["ids"], sp_vals=s["vals"])
        try:
            qp, qi, qv = s["q"]
            sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
                  torch.from_numpy(qv).to(DEV))
            ann.ann_set_launch(ix, "sparse", beam_buffer=buf, beam_list=place)
            r = ann.ann_search_ex(ix, "sparse", sparse=sq, k=10, ef=300, want_stats=True)
            torch.cuda.synchronize()
            got = {k_: v.cpu().numpy() for k_, v in r.items()}
            assert_same(got, oracle.hnsw_search(s["graph"], s["store"], 10, 300, sparse_q=s["q"]))
        finally:
            ix.close()


def test_pq_with_hbm_beam(c1):
    X = c1["X"]
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=4)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(c1["g"], "l2", X.shape[1], x_f32=X, pq_codebook=cb, pq_codes=codes)
    try:
        ref = oracle.hnsw_search(c1["g"], oracle.pq_store(cb, codes, "l2"), 10, 1000, Q=c1["Q"],
                                 rerank_f32=X, rerank=30)
        ann.ann_set_launch(ix, "pq", waves_per_query=2, beam_list="hbm")
        assert_same(gpu(ix, "pq", c1["Q"], 10, 1000, rerank=30), ref)
    finally:
        ix.close()


def test_beam_buffer_bounds(c1):
    for bad in (-2, 1, 63, 4097):
        with pytest.raises(ann.AnnError) as e:
            ann.ann_set_launch(c1["ix"], "f32", beam_buffer=bad)
        assert e.value.code == ann.ANN_EINVAL
    with pytest.raises(ann.AnnError) as e:
        ann.ann_set_launch(c1["ix"], "f32", beam_list=3)
    assert e.value.code == ann.ANN_EINVAL
    assert ann.ann_get_launch(c1["ix"], "f32")["beam_buffer"] == 0
    # an HBM list needs the insert buffer
    ann.ann_set_launch(c1["ix"], "f32", beam_buffer=-1, beam_list="hbm")
    try:
        with pytest.raises(ann.AnnError) as e:
            gpu(c1["ix"], "f32", c1["Q"][:2], 10, 100)
        assert e.value.code == ann.ANN_EINVAL
    finally:
        ann.ann_set_launch(c1["ix"], "f32")
    # a list forced into LDS stops at its size; ANN_EF_MAX bounds the HBM list
    ann.ann_set_launch(c1["ix"], "f32", beam_list="lds")
    try:
        with pytest.raises(ann.AnnError) as e:
            gpu(c1["ix"], "f32", c1["Q"][:2], 10, 21000)
        assert e.value.code == ann.ANN_EBUDGET
    finally:
        ann.ann_set_launch(c1["ix"], "f32")
    with pytest.raises(ann.AnnError) as e:
        gpu(c1["ix"], "f32", c1["Q"][:2], 10, ann.ANN_EF_MAX + 1)
    assert e.value.code == ann.ANN_EBUDGET
