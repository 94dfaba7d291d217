"""Address and undefined-behaviour sanitizer runs on the CPU.

1. The oracle (oracle.cpp) built with -fsanitize=address,undefined runs a
   small workload through every entry point: HNSW build (dense and sparse)
   and search in every representation and key mode, rerank, brute force,
   PQ training / encoding / ADC, IVF training / assignment / search, FP8
   encoding.
2. The library's host code (every csrc/*.hip, sanitizers on the host side
   only) runs what needs no GPU: index-file writing,
   reading and checking, against valid, truncated and corrupted files (the
   reader's input is untrusted), and the description checks of
   ann_index_create's error paths.

Each run is a child process with the sanitizer runtime preloaded; it must
exit cleanly with no sanitizer report.
"""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

REPORT_MARKERS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer",
                  "UndefinedBehaviorSanitizer")


def _run(script, preload, extra_env=None, timeout=600):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": preload,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
                "OMP_NUM_THREADS": "2", "PYTHONPATH": ROOT})
    env.update(extra_env or {})
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True,
                       timeout=timeout, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for m in REPORT_MARKERS:
        assert m not in out, out[-4000:]
    return r.stdout


ORACLE_SCRIPT = r"""
import sys
import numpy as np
import oracle, synth
oracle.LIB_PATH = LIB
for metric in ("l2", "ip"):
    X = synth.gaussian_mixture(0, 600, 16, 4, 0.3)
    Q = synth.gaussian_mixture(0, 7, 16, 4, 0.3, which="queries")
    g = oracle.hnsw_build(X, metric, 8, 32, synth.level_uniforms(0, 600), seq_prefix=100,
                          batch_frac=0.05, batch_cap=64)
    scale = np.abs(X).max(1) / 448
    stores = [oracle.dense_store(X, metric), oracle.dense_store(oracle.to_f16(X), metric, "f16"),
              oracle.dense_store(oracle.to_bf16(X), metric, "bf16")]
    x8, s8 = oracle.encode_fp8_rows(X)
    stores.append(oracle.dense_store(x8, metric, "fp8", fp8_scale=s8))
    sample, init = synth.pq_sample(0, 600, 600, 256)
    cb, _, _ = oracle.pq_train(X, 4, 256, sample, init, max_iter=3)
    codes = oracle.pq_encode(X, cb)
    stores.append(oracle.pq_store(cb, codes, metric))
    for st in stores:
        for kmode in ("canon", "exact"):
            r = oracle.hnsw_search(g, st, 5, 40, Q=Q, kmode=kmode, rerank_f32=X, rerank=12,
                                   want_w=True, visited_cap=600)
            assert r["ids"].shape == (7, 5)
        oracle.bruteforce(st, 600, 5, Q=Q, kmode="canon")
    ks = np.array([1, 3, 5, 2, 5, 4, 1]); efs = np.array([1, 8, 40, 3, 17, 600, 2])
    oracle.hnsw_search(g, stores[0], ks, efs, Q=Q)
    s_ids, s_init = synth.ivf_sample(0, 600, 600, 8)
    cent, _, _ = oracle.ivf_train(X, 8, s_ids, s_init, max_iter=4)
    asg = oracle.ivf_assign(X, cent)
    off, ids = oracle.ivf_lists(asg, 8)
    oracle.ivf_search(stores[1], cent, off, ids, Q, 5, 3, rerank_f32=X, rerank_depth=20)
ip, sid, sv = synth.sparse_zipf(1, 200, 12, vocab=300)
qp, qi, qv = synth.sparse_zipf(1, 5, 6, vocab=300, which="queries")
g = oracle.hnsw_build_sparse(ip, sid, sv, 300, 8, 32, synth.level_uniforms(1, 200))
st = oracle.sparse_store(ip, sid, sv, 300)
for kmode in ("canon", "exact"):
    oracle.hnsw_search(g, st, 5, 30, sparse_q=(qp, qi, qv), kmode=kmode)
oracle.bruteforce(st, 200, 5, sparse_q=(qp, qi, qv))
print("oracle workload done")
"""


def test_oracle_is_clean_under_asan_and_ubsan():
    import oracle
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        flags = [f for f in oracle.CXX_FLAGS if f != "-O2"]
        subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               *flags, oracle.SRC_PATH, "-o", lib])
        out = _run(f"LIB = {lib!r}\n" + ORACLE_SCRIPT, asan)
        assert "oracle workload done" in out


LIBRARY_SCRIPT = r"""
import ctypes as C, os, sys
import numpy as np
sys.modules["torch"] = None          # the host-only library never needs the GPU runtime's torch
import paper_2501_06121_amd as ann
import oracle, synth
ann.LIB_PATH = LIB
L = ann.lib()
X = synth.gaussian_mixture(0, 300, 16, 4, 0.3)
g = oracle.hnsw_build(X, "ip", 8, 32, synth.level_uniforms(0, 300))
sample, init = synth.pq_sample(0, 300, 300, 256)
cb, _, _ = oracle.pq_train(X, 4, 256, sample, init, max_iter=2)
codes = oracle.pq_encode(X, cb)
ip, sid, sv = synth.sparse_zipf(1, 300, 4, vocab=16)   # the vocabulary is d
x8, s8 = oracle.encode_fp8_rows(X)
arrays = dict(x_f32=X, x_f16=oracle.to_f16(X), x_bf16=oracle.to_bf16(X), x_fp8=x8, fp8_scale=s8,
              pq_codebook=cb, pq_codes=codes, sp_indptr=ip, sp_ids=sid, sp_vals=sv)
path = os.path.join(TMP, "ix.bin")
ann.ann_index_save(path, g, "ip", 16, **arrays)
info = ann.ann_index_file_info(path)
assert info["n"] == 300 and info["d"] == 16
data = open(path, "rb").read()
rng = np.random.default_rng(0)
bad = os.path.join(TMP, "bad.bin")
def check(blob):
    with open(bad, "wb") as f:
        f.write(blob)
    rc = L.ann_index_file_info(os.fsencode(bad), C.byref(ann.AnnIndexInfo()))
    assert rc in (ann.ANN_OK, ann.ANN_EFORMAT), rc
    return rc
n_ok = 0
# truncations, at every section boundary region and at random lengths
for cut in list(range(0, 200, 7)) + list(rng.integers(0, len(data), 60)):
    assert check(data[:int(cut)]) == ann.ANN_EFORMAT
# single-byte corruptions anywhere, header bytes included
for pos in list(range(0, 256)) + list(rng.integers(0, len(data), 300)):
    b = bytearray(data)
    b[int(pos)] ^= 1 << int(rng.integers(0, 8))
    n_ok += check(bytes(b)) == ann.ANN_OK
# random garbage of header size and beyond
for size in (0, 1, 127, 128, 129, 4096):
    check(rng.integers(0, 256, size, dtype=np.uint8).tobytes())
# a valid header over a huge claimed section table
b = bytearray(data); b[12:16] = (1 << 30).to_bytes(4, "little")
check(bytes(b))
# description errors of ann_index_create are caught before any device work
D, keep = ann._desc(g, "ip", 16, x_f32=X)
for field, value in (("n", -1), ("d", 0), ("M0", 0), ("entry_point", 10 ** 6), ("max_level", 99)):
    saved = getattr(D, field)
    setattr(D, field, value)
    rc = L.ann_index_save(C.byref(D), os.fsencode(bad))
    assert rc != ann.ANN_OK, (field, value)
    setattr(D, field, saved)
assert n_ok == 0, n_ok     # every flipped bit is caught (checksums, zero padding)
print("library host workload done")
"""


def test_library_host_code_is_clean_under_asan_and_ubsan():
    hipcc = "/opt/rocm/bin/hipcc"
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    from paper_2501_06121_amd import build as hip_build
    srcs = hip_build.sources()
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        procs = []
        for s in srcs:
            o = os.path.join(tmp, os.path.basename(s) + ".o")
            objs.append(o)
            # device code as usual; the sanitizers apply to the host side alone
            cmd = [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                   "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer",
                   "-Wno-unused-result", "-Wno-unused-value",
                   f"-I{hip_build.INCLUDE}", f"-I{hip_build.CSRC}", "-c", s, "-o", o]
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                          text=True))
        for p in procs:
            _, err = p.communicate()
            assert p.returncode == 0, err[-3000:]
        lib = os.path.join(tmp, "libann_san.so")
        hip_rt = hip_build.hip_runtime_dir()
        # the sanitizer runtime is preloaded into the child process, which
        # resolves the instrumentation's symbols
        subprocess.check_call(["g++", "-shared", "-fPIC", "-o", lib, *objs, f"-L{hip_rt}",
                               "-l:libamdhip64.so", f"-Wl,-rpath,{hip_rt}", "-lpthread"])
        out = _run(f"LIB = {lib!r}\nTMP = {tmp!r}\n" + LIBRARY_SCRIPT, rt[0])
        assert "library host workload done" in out
