"""Parity at full size: 1,000,000 x 768 vMF, inner product, HNSW M=32.

The GPU searches all 10,000 queries in one launch, in the configuration the
benchmark times; sampled queries are then checked one by one against the
oracle (same graph, same representation, same ef), bit for bit.  Skipped when
the oracle-built graph (data/vmf1m) is not present.
"""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "data", "vmf1m")


def say(*a):
    print("[parity-1m]", *a, flush=True)


@pytest.fixture(scope="module")
def big():
    gpath = os.path.join(DATA, "graph.npz")
    if not os.path.exists(gpath):
        pytest.skip("data/vmf1m/graph.npz not built (python -m oracle.build_index vmf1m)")
    g = oracle.Graph.load(gpath)
    spec = synth.WORKLOADS["vmf1m"]
    say("regenerating 1M x 768")
    X = synth.dense_base(spec)
    Q = synth.dense_queries(spec)
    X16 = X.astype(np.float16).view(np.uint16)   # equals oracle.to_f16 (pinned on the CPU)
    f8, s8 = oracle.encode_fp8_rows(X)
    cb = codes = None
    if os.path.exists(os.path.join(DATA, "pq.npz")):
        z = np.load(os.path.join(DATA, "pq.npz"))
        cb, codes = z["codebook"], z["codes"]
    say("uploading")
    ix = ann.ann_index_create(g, "ip", X.shape[1], x_f32=X, x_f16=X16, x_fp8=f8, fp8_scale=s8,
                              pq_codebook=cb, pq_codes=codes)
    gt = None
    if os.path.exists(os.path.join(DATA, "gt.npz")):
        gt = np.load(os.path.join(DATA, "gt.npz"))["ids"]
    yield dict(g=g, X=X, X16=X16, f8=f8, s8=s8, cb=cb, codes=codes, Q=Q, ix=ix, gt=gt)
    ix.close()


def bench_ef():
    import json
    p = os.path.join(ROOT, "profiles", "vmf1m_ef_sweep.json")
    if not os.path.exists(p):
        return 256, 256
    s = json.load(open(p))

    def pick(key):
        pts = sorted(s[key], key=lambda r: r["ef"])
        for r in pts:
            if r["recall"] >= 0.95:
                return r["ef"]
        return pts[-1]["ef"]
    return pick("f16+rerank"), pick("f32")


@pytest.mark.parametrize("mode", ["f16", "f32"])
def test_full_batch_sampled_bitexact(big, mode):
    ef16, ef32 = bench_ef()
    ef, rr = (ef16, 40) if mode == "f16" else (ef32, 0)
    say(mode, "ef", ef, "all 10,000 queries on the GPU")
    q = torch.from_numpy(big["Q"]).to("cuda:0")
    r = ann.ann_search_ex(big["ix"], mode, queries=q, k=10, ef=ef, rerank=rr, want_stats=True)
    torch.cuda.synchronize()
    ids, dists, stats = (r[k].cpu().numpy() for k in ("ids", "dists", "stats"))
    assert np.all(r["status"].cpu().numpy() == 0)
    sample = np.random.default_rng(0).choice(big["Q"].shape[0], 48, replace=False)
    st = oracle.dense_store(big["X16"], "ip", "f16") if mode == "f16" else oracle.dense_store(big["X"], "ip")
    say("oracle on", len(sample), "sampled queries")
    ref = oracle.hnsw_search(big["g"], st, 10, ef, Q=big["Q"][sample],
                             rerank_f32=big["X"] if rr else None, rerank=rr)
    assert np.array_equal(ids[sample], ref["ids"])
    assert np.array_equal(dists[sample], ref["keys"])
    assert np.array_equal(stats[sample, 1], ref["stats"][:, 2])
    assert np.array_equal(stats[sample, 2], ref["stats"][:, 3])
    # distances agree with the FP64 evaluation within 1e-5 relative
    ex = oracle.keys(oracle.dense_store(big["X"], "ip"), big["Q"][sample], ref["ids"], "exact")
    if mode == "f32" or rr:
        assert np.all(np.abs(dists[sample] - ex) <= 1e-5 * np.abs(ex) + 1e-7)
    if big["gt"] is not None:
        rec_all = oracle.recall_at_k(ids, big["gt"], 10)
        rec_s = oracle.recall_at_k(ids[sample], big["gt"][sample], 10)
        say(mode, "recall@10 all", rec_all, "sample", rec_s)
        assert abs(oracle.recall_at_k(ref["ids"], big["gt"][sample], 10) - rec_s) <= 0.002


def test_maximum_ef(big):
    ef = ann.ANN_EF_MAX
    say("ef =", ef, "on 6 queries")
    Q = big["Q"][:6]
    r = ann.ann_search_ex(big["ix"], "f16", queries=torch.from_numpy(Q).to("cuda:0"), k=10,
                          ef=ef, rerank=40, want_stats=True)
    torch.cuda.synchronize()
    ref = oracle.hnsw_search(big["g"], oracle.dense_store(big["X16"], "ip", "f16"), 10, ef, Q=Q,
                             rerank_f32=big["X"], rerank=40)
    assert np.array_equal(r["ids"].cpu().numpy(), ref["ids"])
    assert np.array_equal(r["stats"].cpu().numpy()[:, 2], ref["stats"][:, 3])


@pytest.mark.parametrize("mode", ["pq", "fp8"])
def test_quantized_traversal_with_rerank(big, mode):
    """PQ (64 x 256, ADC tables in LDS) and FP8-E4M3 traversal, FP32 rerank of
    the first 100 beam entries, on the graph built on the FP32 originals."""
    if mode == "pq" and big["codes"] is None:
        pytest.skip("data/vmf1m/pq.npz not built (python -m oracle.build_index vmf1m --what pq)")
    ef = 400
    say(mode, "ef", ef, "rerank 100, all 10,000 queries")
    q = torch.from_numpy(big["Q"]).to("cuda:0")
    r = ann.ann_search_ex(big["ix"], mode, queries=q, k=10, ef=ef, rerank=100, want_stats=True)
    torch.cuda.synchronize()
    ids, dists, stats = (r[k].cpu().numpy() for k in ("ids", "dists", "stats"))
    sample = np.random.default_rng(1).choice(big["Q"].shape[0], 32, replace=False)
    if mode == "pq":
        st = oracle.pq_store(big["cb"], big["codes"], "ip")
    else:
        st = oracle.dense_store(big["f8"], "ip", "fp8", fp8_scale=big["s8"])
    ref = oracle.hnsw_search(big["g"], st, 10, ef, Q=big["Q"][sample], rerank_f32=big["X"],
                             rerank=100)
    assert np.array_equal(ids[sample], ref["ids"])
    assert np.array_equal(dists[sample], ref["keys"])
    assert np.array_equal(stats[sample, 2], ref["stats"][:, 3])
    if big["gt"] is not None:
        say(mode, "recall@10", oracle.recall_at_k(ids, big["gt"], 10))


def test_pq_training_and_encoding_at_full_size(big):
    """PQ 64 x 256 trained on the device with the oracle's sample, init and
    iteration budget (100,000 sample rows, 25 iterations) equals the oracle's
    stored codebook bit for bit, and the device codes of all 1,000,000 rows
    equal the oracle's stored codes."""
    if big["codes"] is None:
        pytest.skip("data/vmf1m/pq.npz not built")
    X = torch.from_numpy(big["X"]).to("cuda:0")
    sample, init = synth.pq_sample(0, big["X"].shape[0], 100_000, 256)
    import time
    say("pq training on the device, 100,000 sample rows, 25 iterations")
    t = time.perf_counter()
    cb, iters = ann.ann_pq_train(X, torch.from_numpy(sample).to("cuda:0"),
                                 torch.from_numpy(init).to("cuda:0"), 64, 256, 25)
    torch.cuda.synchronize()
    say(f"trained in {time.perf_counter() - t:.3f} s ({iters} iterations)")
    assert np.array_equal(cb.cpu().numpy().view(np.uint32), big["cb"].view(np.uint32))
    say("pq encoding of 1,000,000 rows")
    cbd = torch.from_numpy(big["cb"]).to("cuda:0")
    t = time.perf_counter()
    codes = ann.ann_pq_encode(X, cbd)
    torch.cuda.synchronize()
    say(f"encoded in {time.perf_counter() - t:.3f} s")
    assert np.array_equal(codes.cpu().numpy(), big["codes"])


def test_graph_build_at_full_size(big):
    """HNSW construction of the 1M x 768 set on the device (M=32, efC=200,
    2,000 nodes one at a time, then batches of 2% up to 2,048) equals the
    oracle's stored graph: levels, every list in order, entry point."""
    import time
    X = torch.from_numpy(big["X"]).to("cuda:0")
    u = synth.level_uniforms(0, big["X"].shape[0])
    say("graph construction on the device, 1,000,000 x 768")
    t = time.perf_counter()
    g = ann.ann_hnsw_build(X, "ip", 32, 200, u, seq_prefix=2000, batch_frac=0.02, batch_cap=2048)
    say(f"built in {time.perf_counter() - t:.1f} s")
    ref = big["g"]
    assert g.max_level == ref.max_level and g.entry == ref.entry
    assert np.array_equal(g.levels, ref.levels)
    assert np.array_equal(g.upper_off, ref.upper_off)
    assert np.array_equal(g.upper_adj, ref.upper_adj)
    assert np.array_equal(g.adj0, ref.adj0)


def ivf_nprobe():
    import json
    p = os.path.join(ROOT, "profiles", "vmf1m_ivf_sweep.json")
    if not os.path.exists(p):
        return 64, 64
    s = json.load(open(p))

    def pick(key):
        pts = sorted(s[key], key=lambda r: r["nprobe"])
        for r in pts:
            if r["recall"] >= 0.95:
                return r["nprobe"]
        return pts[-1]["nprobe"]
    return pick("f16+rerank"), pick("f32")


@pytest.mark.parametrize("mode", ["f16", "f32"])
def test_ivf_full_batch_sampled_bitexact(big, mode):
    """IVF over the oracle's 1,024 lists: all 10,000 queries in one launch at the
    benchmark's nprobe; 24 sampled queries checked against the oracle."""
    zp = os.path.join(DATA, "ivf.npz")
    if not os.path.exists(zp):
        pytest.skip("data/vmf1m/ivf.npz not built (python -m oracle.build_index vmf1m --what ivf)")
    z = np.load(zp)
    np16, np32 = ivf_nprobe()
    npb, rr = (np16, 40) if mode == "f16" else (np32, 0)
    v = ann.ann_ivf_create(big["ix"], z["centroids"], z["list_off"], z["list_ids"])
    try:
        say("ivf", mode, "nprobe", npb, "all 10,000 queries on the GPU")
        q = torch.from_numpy(big["Q"]).to("cuda:0")
        r = ann.ann_ivf_search(v, q, 10, npb, mode=mode, rerank=rr, want_probes=True, want_stats=True)
        torch.cuda.synchronize()
        got = {k_: t.cpu().numpy() for k_, t in r.items()}
    finally:
        v.close()
    sample = np.random.default_rng(5).choice(big["Q"].shape[0], 24, replace=False)
    st = oracle.dense_store(big["X16"], "ip", "f16") if mode == "f16" else oracle.dense_store(big["X"], "ip")
    ref = oracle.ivf_search(st, z["centroids"], z["list_off"], z["list_ids"], big["Q"][sample], 10, npb,
                            rerank_f32=big["X"] if rr else None, rerank_depth=rr)
    assert np.array_equal(got["probes"][sample], ref["probes"])
    assert np.array_equal(got["stats"][sample], ref["stats"])
    assert np.array_equal(got["ids"][sample], ref["ids"])
    assert np.array_equal(got["dists"][sample], ref["keys"])
    if big["gt"] is not None:
        rec = oracle.recall_at_k(got["ids"], big["gt"], 10)
        say(f"ivf {mode} recall@10 {rec:.4f}")
        assert rec >= 0.95


def test_ivf_training_and_assignment_at_full_size(big):
    """The device trains the 1,024 coarse centroids on the 100,000-row sample and
    assigns all 1,000,000 rows, equal to the oracle's stored index."""
    zp = os.path.join(DATA, "ivf.npz")
    if not os.path.exists(zp):
        pytest.skip("data/vmf1m/ivf.npz not built (python -m oracle.build_index vmf1m --what ivf)")
    import time
    z = np.load(zp)
    nlist = z["centroids"].shape[0]
    sample, init = synth.ivf_sample(0, big["X"].shape[0], 100_000, nlist)
    Xd = torch.from_numpy(big["X"]).to("cuda:0")
    t = time.perf_counter()
    cent, iters = ann.ann_ivf_train(Xd, torch.from_numpy(sample).to("cuda:0"),
                                    torch.from_numpy(init).to("cuda:0"), nlist, max_iter=25)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    asg = ann.ann_ivf_assign(Xd, cent)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say(f"ivf trained in {t1 - t:.2f} s ({iters} iterations), 1M rows assigned in {t2 - t1:.3f} s")
    assert iters == int(z["iters"])
    assert np.array_equal(cent.cpu().numpy(), z["centroids"])
    off, ids = ann.ann_ivf_group(asg.cpu().numpy(), nlist)
    assert np.array_equal(off, z["list_off"]) and np.array_equal(ids, z["list_ids"])
