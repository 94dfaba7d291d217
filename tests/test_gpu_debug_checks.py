"""The search kernels' beam invariants, checked on the device.

libann_debug.so is the library built with ANN_DEBUG_CHECKS: between
expansions every workgroup checks that its sorted list and insert buffer are
strictly ascending in (key, id), |W| <= ef after the cut, every id is in
[0, n), every entry before the scan position is expanded and the candidate
counts fit, and sets flag bits on a violation (never a trap).  A child
process loads it (the test process holds the regular library) and runs
every beam layout, storage mode, mixed k/ef and the server; the flags must
stay zero and the results must still equal the oracle's.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_2501_06121_amd", "libann_debug.so")

pytestmark = pytest.mark.gpu

SCRIPT = r"""
import sys
import numpy as np
import torch
import oracle, synth
import paper_2501_06121_amd as ann
ann.LIB_PATH = LIB
DEV = "cuda:0"

def say(*a):
    print(*a, flush=True)

def check(ix, tag):
    f = ann.ann_debug_flags(ix)
    assert f == 0, f"{tag}: invariant flags {f:#x}"

# dense L2, 4,000 x 64
n, d = 4000, 64
X = synth.gaussian_mixture(7, n, d, 16, 0.3)
Q = synth.gaussian_mixture(7, 24, d, 16, 0.3, which="queries")
g = oracle.hnsw_build(X, "l2", 16, 64, synth.level_uniforms(7, n))
f8, s8 = oracle.encode_fp8_rows(X)
sample, init = synth.pq_sample(7, n, n, 256)
cb, _, _ = oracle.pq_train(X, 8, 256, sample, init, max_iter=2)
codes = oracle.pq_encode(X, cb)
ix = ann.ann_index_create(g, "l2", d, x_f32=X, x_f16=oracle.to_f16(X), x_bf16=oracle.to_bf16(X),
                          x_fp8=f8, fp8_scale=s8, pq_codebook=cb, pq_codes=codes)
q = torch.from_numpy(Q).to(DEV)
stores = {"f32": oracle.dense_store(X, "l2"),
          "f16": oracle.dense_store(oracle.to_f16(X), "l2", "f16"),
          "bf16": oracle.dense_store(oracle.to_bf16(X), "l2", "bf16"),
          "fp8": oracle.dense_store(f8, "l2", "fp8", fp8_scale=s8),
          "pq": oracle.pq_store(cb, codes, "l2")}
layouts = [dict(), dict(beam_buffer=64), dict(beam_buffer=200), dict(beam_list="hbm"),
           dict(beam_buffer=64, beam_list="hbm"), dict(beam_buffer=-1, beam_list="lds")]
for mode, st in stores.items():
    refs = {ef: oracle.hnsw_search(g, st, 10, ef, Q=Q, rerank_f32=X, rerank=20)["ids"]
            for ef in (10, 300, 1500)}
    for lay in layouts:
        for waves in (1, 4):
            ann.ann_set_launch(ix, mode, waves_per_query=waves, **lay)
            for ef in (10, 300, 1500):
                try:
                    r = ann.ann_search_ex(ix, mode, queries=q, k=10, ef=ef, rerank=20)
                except ann.AnnError as e:
                    if e.code == ann.ANN_EBUDGET:
                        continue          # this layout does not fit this ef on chip
                    raise
                torch.cuda.synchronize()
                assert np.array_equal(r["ids"].cpu().numpy(), refs[ef]), (mode, lay, waves, ef)
                check(ix, f"{mode} {lay} waves {waves} ef {ef}")
        ann.ann_set_launch(ix, mode)
    say("mode", mode, "ok")
# mixed k and ef in one launch
rng = np.random.default_rng(3)
ks = rng.choice([1, 10, 100], Q.shape[0]).astype(np.int32)
efs = rng.choice([16, 100, 1500, 3000], Q.shape[0]).astype(np.int32)
r = ann.ann_search_ex(ix, "f32", queries=q, k=torch.from_numpy(ks).to(DEV),
                      ef=torch.from_numpy(efs).to(DEV), k_max=100, ef_max=3000)
torch.cuda.synchronize()
ref = oracle.hnsw_search(g, stores["f32"], ks, efs, Q=Q)
assert np.array_equal(r["ids"].cpu().numpy(), ref["ids"])
check(ix, "mixed k/ef")
# the server's kernel
srv = ann.Server(ix, mode="f16", rerank=20, max_inflight=64, k_max=100, ef_max=512)
for i in range(40):
    assert srv.submit(i, Q[i % Q.shape[0]], [10, 100][i % 2], [64, 512][i % 3 == 0])
got = 0
import time
t = time.time()
while got < 40 and time.time() - t < 60:
    got += len(srv.poll())
srv.close()
assert got == 40
check(ix, "server")
ix.close()
say("dense ok")

# sparse rows
ip, sid, sv = synth.sparse_zipf(2, 2000, 20, vocab=500)
qp, qi, qv = synth.sparse_zipf(2, 16, 8, vocab=500, which="queries")
gs = oracle.hnsw_build_sparse(ip, sid, sv, 500, 8, 32, synth.level_uniforms(2, 2000))
ixs = ann.ann_index_create(gs, "ip", 500, sp_indptr=ip, sp_ids=sid, sp_vals=sv)
sq = (torch.from_numpy(qp).to(DEV), torch.from_numpy(qi.view(np.int16)).to(DEV),
      torch.from_numpy(qv).to(DEV))
sts = oracle.sparse_store(ip, sid, sv, 500)
for lay in layouts[:4]:
    ann.ann_set_launch(ixs, "sparse", **lay)
    for ef in (10, 300, 1500):
        r = ann.ann_search_ex(ixs, "sparse", sparse=sq, k=10, ef=ef)
        torch.cuda.synchronize()
        ref = oracle.hnsw_search(gs, sts, 10, ef, sparse_q=(qp, qi, qv))
        assert np.array_equal(r["ids"].cpu().numpy(), ref["ids"]), (lay, ef)
        check(ixs, f"sparse {lay} ef {ef}")
ixs.close()
say("sparse ok")
print("debug checks clean", flush=True)
"""


def test_beam_invariants_hold_in_every_layout_and_mode():
    if not os.path.exists(DEBUG_LIB):
        pytest.fail(f"{DEBUG_LIB} is missing: build it with paper_2501_06121_amd.build.build_debug()")
    print("debug-checks library in a child process", flush=True)
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-u", "-c", f"LIB = {DEBUG_LIB!r}\n" + SCRIPT], env=env,
                       capture_output=True, text=True, timeout=280, cwd=ROOT)
    out = r.stdout + r.stderr
    print(out[-3000:], flush=True)
    assert r.returncode == 0, out[-4000:]
    assert "debug checks clean" in r.stdout


def test_regular_library_reports_no_checks():
    torch = pytest.importorskip("torch")
    import numpy as np
    import oracle
    import paper_2501_06121_amd as ann
    X = np.random.default_rng(0).standard_normal((50, 16)).astype(np.float32)
    g = oracle.hnsw_build(X, "l2", 4, 8, np.zeros(50))
    ix = ann.ann_index_create(g, "l2", 16, x_f32=X)
    try:
        with pytest.raises(ann.AnnError) as e:
            ann.ann_debug_flags(ix)
        assert e.value.code == ann.ANN_EUNSUP
    finally:
        ix.close()
    assert torch is not None
