"""Indexes loaded from files: the oracle writes the file, the library loads
it onto the GPU, and every representation in it searches exactly like the
oracle's search of the same arrays.  A device-built graph saved by the
library and loaded back searches like the one it came from."""
import numpy as np
import pytest

import oracle
import oracle.index_file as oif
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-index-file]", *a, flush=True)


def search(ix, mode, Q, k, ef, rerank=0, sparse=None):
    if sparse is not None:
        qp, qi, qv = sparse
        sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
              torch.from_numpy(qv).to(DEV))
        r = ann.ann_search_ex(ix, mode, sparse=sq, k=k, ef=ef, want_stats=True)
    else:
        r = ann.ann_search_ex(ix, mode, queries=torch.from_numpy(Q).to(DEV), k=k, ef=ef,
                              rerank=rerank, want_stats=True)
    torch.cuda.synchronize()
    return {k_: v.cpu().numpy() for k_, v in r.items()}


def test_oracle_written_dense_file(tmp_path, gmm10k):
    X, Q, g = gmm10k["X"], gmm10k["Q"], gmm10k["graph"]
    f8, s8 = oracle.encode_fp8_rows(X)
    sample, init = synth.pq_sample(0, X.shape[0], 5000, 256)
    cb, _, _ = oracle.pq_train(X, 16, 256, sample, init, max_iter=4)
    codes = oracle.pq_encode(X, cb)
    arrays = dict(x_f32=X, x_f16=oracle.to_f16(X), x_bf16=oracle.to_bf16(X), x_fp8=f8,
                  fp8_scale=s8, pq_codebook=cb, pq_codes=codes)
    path = tmp_path / "gmm10k.idx"
    oif.write(path, g, "l2", X.shape[1], **arrays)
    say("load", path)
    ix = ann.ann_index_load(str(path))
    try:
        info = ix.info()
        assert (info["n"], info["d"], info["entry_point"], info["max_level"]) == \
            (g.n, 128, g.entry, g.max_level)
        stores = {"f32": oracle.dense_store(X, "l2"),
                  "f16": oracle.dense_store(oracle.to_f16(X), "l2", "f16"),
                  "bf16": oracle.dense_store(oracle.to_bf16(X), "l2", "bf16"),
                  "fp8": oracle.dense_store(f8, "l2", "fp8", fp8_scale=s8),
                  "pq": oracle.pq_store(cb, codes, "l2")}
        for mode, st in stores.items():
            rr = 0 if mode == "f32" else 30
            say("mode", mode, "rerank", rr)
            got = search(ix, mode, Q, 10, 80, rerank=rr)
            ref = oracle.hnsw_search(g, st, 10, 80, Q=Q, rerank_f32=X if rr else None, rerank=rr)
            assert np.array_equal(got["ids"], ref["ids"]), mode
            assert np.array_equal(got["dists"], ref["keys"]), mode
            assert np.array_equal(got["stats"][:, 2], ref["stats"][:, 3]), mode
    finally:
        ix.close()


def test_oracle_written_sparse_file(tmp_path, sparse_small):
    s = sparse_small
    path = tmp_path / "sparse.idx"
    oif.write(path, s["graph"], "ip", s["vocab"], sp_indptr=s["indptr"], sp_ids=s["ids"],
              sp_vals=s["vals"])
    ix = ann.ann_index_load(str(path))
    try:
        got = search(ix, "sparse", None, 10, 100, sparse=s["q"])
    finally:
        ix.close()
    ref = oracle.hnsw_search(s["graph"], s["store"], 10, 100, sparse_q=s["q"])
    assert np.array_equal(got["ids"], ref["ids"])
    assert np.array_equal(got["dists"], ref["keys"])


def test_device_built_graph_saved_and_loaded(tmp_path, vmf_small):
    X, Q = vmf_small["X"], vmf_small["Q"]
    n = X.shape[0]
    say("device build", n, "x 768")
    bg = ann.ann_hnsw_build(torch.from_numpy(X).to(DEV), "ip", 16, 64, synth.level_uniforms(9, n),
                            seq_prefix=500, batch_frac=0.02, batch_cap=128)
    path = tmp_path / "built.idx"
    ann.ann_index_save(str(path), bg, "ip", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X))
    h, arrs = oif.read(path)        # the oracle reads what the library wrote
    assert np.array_equal(arrs["adj0"], bg.adj0) and h["entry_point"] == bg.entry
    a = ann.ann_index_create(bg, "ip", X.shape[1], x_f32=X, x_f16=oracle.to_f16(X))
    b = ann.ann_index_load(str(path))
    try:
        for mode, rr in (("f32", 0), ("f16", 40)):
            ra = search(a, mode, Q, 10, 100, rerank=rr)
            rb = search(b, mode, Q, 10, 100, rerank=rr)
            assert np.array_equal(ra["ids"], rb["ids"]) and np.array_equal(ra["dists"], rb["dists"])
    finally:
        a.close()
        b.close()
