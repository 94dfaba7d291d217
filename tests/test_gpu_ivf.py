"""GPU parity of the IVF index: probes, scanned rows, keys and ids of the HIP
path against the CPU oracle's IVF search on the same seeded inputs.

Probe keys and row keys are evaluated in the same fixed FP32 order on both
sides, so the probe lists, the evaluation counts, the ids and the keys must
agree exactly.
"""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[gpu-ivf]", *a, flush=True)


def coarse(X, nlist, seed=0, iters=10):
    sample, init = synth.ivf_sample(seed, X.shape[0], min(X.shape[0], 20 * nlist), nlist)
    cent, _, _ = oracle.ivf_train(X, nlist, sample, init, max_iter=iters)
    off, ids = oracle.ivf_lists(oracle.ivf_assign(X, cent), nlist)
    return cent, off, ids


@pytest.fixture(scope="module")
def l2set(gmm10k):
    X, g = gmm10k["X"], gmm10k["graph"]
    f8, s8 = oracle.encode_fp8_rows(X)
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=6)
    codes = oracle.pq_encode(X, cb)
    ix = ann.ann_index_create(g, "l2", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X),
                              x_bf16=oracle.to_bf16(X), x_fp8=f8, fp8_scale=s8,
                              pq_codebook=cb, pq_codes=codes)
    cent, off, ids = coarse(X, 64)
    v = ann.ann_ivf_create(ix, cent, off, ids)
    yield dict(ix=ix, ivf=v, X=X, Q=gmm10k["Q"], f8=f8, s8=s8, cb=cb, codes=codes, cent=cent,
               off=off, ids=ids, metric="l2")
    v.close()
    ix.close()


@pytest.fixture(scope="module")
def ipset(vmf_small):
    X, g = vmf_small["X"], vmf_small["graph"]
    f8, s8 = oracle.encode_fp8_rows(X)
    ix = ann.ann_index_create(g, "ip", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X),
                              x_bf16=oracle.to_bf16(X), x_fp8=f8, fp8_scale=s8)
    cent, off, ids = coarse(X, 40)
    v = ann.ann_ivf_create(ix, cent, off, ids)
    yield dict(ix=ix, ivf=v, X=X, Q=vmf_small["Q"], f8=f8, s8=s8, cent=cent, off=off, ids=ids,
               metric="ip")
    v.close()
    ix.close()


def store_for(s, mode):
    X, metric = s["X"], s["metric"]
    if mode == "f32":
        return oracle.dense_store(X, metric)
    if mode == "f16":
        return oracle.dense_store(oracle.to_f16(X), metric, "f16")
    if mode == "bf16":
        return oracle.dense_store(oracle.to_bf16(X), metric, "bf16")
    if mode == "fp8":
        return oracle.dense_store(s["f8"], metric, "fp8", fp8_scale=s["s8"])
    return oracle.pq_store(s["cb"], s["codes"], metric)


def run(s, mode, Q, k, nprobe, rerank=0, ivf=None, group=0):
    q = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    r = ann.ann_ivf_search(ivf or s["ivf"], q, k, nprobe, mode=mode, rerank=rerank,
                           want_probes=True, want_stats=True, group=group)
    torch.cuda.synchronize()
    return {k_: t.cpu().numpy() for k_, t in r.items()}


def check(s, mode, k, nprobe, rerank=0, Q=None, group=0):
    Q = s["Q"] if Q is None else Q
    ref = oracle.ivf_search(store_for(s, mode), s["cent"], s["off"], s["ids"], Q, k, nprobe,
                            rerank_f32=s["X"] if rerank else None, rerank_depth=rerank)
    got = run(s, mode, Q, k, nprobe, rerank, group=group)
    assert np.array_equal(got["probes"], ref["probes"]), np.argwhere(got["probes"] != ref["probes"])[:5]
    assert np.array_equal(got["stats"], ref["stats"])
    assert np.array_equal(got["ids"], ref["ids"]), np.argwhere(got["ids"] != ref["ids"])[:5]
    assert np.array_equal(got["dists"], ref["keys"])
    return got


@pytest.mark.parametrize("mode", ["f32", "f16", "bf16", "fp8", "pq"])
@pytest.mark.parametrize("nprobe", [1, 6, 64])
@pytest.mark.parametrize("group", [0, 1])
def test_l2_modes_bitexact(l2set, mode, nprobe, group):
    # group 0: the default (the shared scan for the dense modes); 1: one query per workgroup
    say("ivf l2 gmm10k", mode, "nprobe", nprobe, "group", group)
    check(l2set, mode, 10, nprobe, group=group)


@pytest.mark.parametrize("mode", ["f32", "f16", "bf16", "fp8"])
@pytest.mark.parametrize("group", [1, 3, 8, 16])
def test_ip_768_modes_bitexact(ipset, mode, group):
    # 64 queries: groups of 3 leave a ragged last workgroup
    say("ivf ip 4096 x 768", mode, "group", group)
    check(ipset, mode, 10, 5, group=group)


@pytest.mark.parametrize("group", [2, 5, 8, 13])
def test_shared_scan_with_rerank_and_large_k(ipset, group):
    say("ivf shared scan, rerank 40 and k 300, group", group)
    check(ipset, "f16", 10, 9, rerank=40, group=group)
    check(ipset, "bf16", 300, 3, group=group)


@pytest.mark.parametrize("mode,rerank", [("f16", 40), ("bf16", 40), ("pq", 100), ("fp8", 100)])
def test_rerank_bitexact(l2set, mode, rerank):
    say("ivf rerank", mode, rerank)
    check(l2set, mode, 10, 8, rerank=rerank)


def test_ip_rerank_bitexact(ipset):
    say("ivf ip rerank f16 40")
    check(ipset, "f16", 10, 7, rerank=40)


@pytest.mark.parametrize("k", [1, 100, 1024])
def test_k_range(l2set, k):
    say("ivf k", k)
    check(l2set, "f16", k, 4)


def test_nprobe_above_nlist_scans_everything(l2set):
    say("ivf nprobe 100 > nlist 64")
    got = check(l2set, "f32", 10, 100)
    assert np.all(got["stats"][:, 0] == l2set["X"].shape[0])
    assert np.all(got["probes"][:, 64:] == -1)
    bi, bk = oracle.bruteforce(oracle.dense_store(l2set["X"], "l2"), l2set["X"].shape[0], 10,
                               Q=l2set["Q"], kmode="canon")
    assert np.array_equal(got["ids"], bi) and np.array_equal(got["dists"], bk)


def test_padding_and_empty_lists(l2set):
    # 200 centroids over a 10k set with 32 mixture centres: many lists are
    # small or empty; one probe of a small list leaves padding
    X = l2set["X"]
    cent, off, ids = coarse(X, 200, seed=3, iters=3)
    sizes = np.diff(off)
    v = ann.ann_ivf_create(l2set["ix"], cent, off, ids)
    try:
        s = dict(l2set, ivf=v, cent=cent, off=off, ids=ids)
        say("ivf padding: empty lists", int((sizes == 0).sum()), "min nonempty", int(sizes[sizes > 0].min()))
        got = check(s, "f32", 64, 1)
        assert (got["ids"] == -1).any()
        check(s, "f16", 20, 3, rerank=30)
    finally:
        v.close()


def test_batches_and_streams(l2set):
    # nq = 0, one query, and a batch on a side stream without the probe output
    q = torch.from_numpy(l2set["Q"]).to(DEV)
    r = ann.ann_ivf_search(l2set["ivf"], q[:0], 10, 4, mode="f16")
    assert r["ids"].shape == (0, 10)
    check(l2set, "f16", 10, 4, Q=l2set["Q"][:1])
    ref = oracle.ivf_search(store_for(l2set, "f16"), l2set["cent"], l2set["off"], l2set["ids"],
                            l2set["Q"], 10, 4)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        r = ann.ann_ivf_search(l2set["ivf"], q, 10, 4, mode="f16", stream=st)
    st.synchronize()
    assert np.array_equal(r["ids"].cpu().numpy(), ref["ids"])
    assert np.array_equal(r["dists"].cpu().numpy(), ref["keys"])


def test_bad_arguments(l2set):
    q = torch.from_numpy(l2set["Q"]).to(DEV)
    for kw, code in ((dict(k=0), ann.ANN_EINVAL), (dict(k=ann.ANN_K_MAX + 1), ann.ANN_EINVAL),
                     (dict(nprobe=0), ann.ANN_EINVAL), (dict(mode="sparse"), ann.ANN_EUNSUP),
                     (dict(rerank=ann.ANN_K_MAX + 1), ann.ANN_EINVAL),
                     (dict(group=17), ann.ANN_EINVAL), (dict(group=-1), ann.ANN_EINVAL),
                     (dict(mode="pq", group=2), ann.ANN_EINVAL)):
        args = dict(k=10, nprobe=4, mode="f16")
        args.update(kw)
        with pytest.raises(ann.AnnError) as e:
            ann.ann_ivf_search(l2set["ivf"], q, args["k"], args["nprobe"], mode=args["mode"],
                               rerank=args.get("rerank", 0), group=args.get("group", 0))
        assert e.value.code == code, kw
    cent, off, ids = l2set["cent"], l2set["off"], l2set["ids"]
    bad = ids.copy()
    bad[5] = bad[6]
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_create(l2set["ix"], cent, off, bad)
    assert e.value.code == ann.ANN_EFORMAT
    bad_off = off.copy()
    bad_off[-1] -= 1
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_create(l2set["ix"], cent, bad_off, ids)
    assert e.value.code == ann.ANN_EFORMAT


def test_default_group_falls_back_when_the_shared_layout_does_not_fit(l2set):
    # k = rerank = 1024 with every list probed: eight 1024-entry lists per
    # workgroup do not fit beside a tile, so the default takes one query per
    # workgroup, and an explicit group of 8 is refused
    say("ivf k 1024 rerank 1024 nprobe 64 (default group)")
    check(l2set, "f16", 1024, 64, rerank=1024, Q=l2set["Q"][:20])
    q = torch.from_numpy(l2set["Q"][:20]).to(DEV)
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_search(l2set["ivf"], q, 1024, 64, mode="f16", rerank=1024, group=8)
    assert e.value.code == ann.ANN_EBUDGET
