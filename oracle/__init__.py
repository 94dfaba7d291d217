"""CPU oracle for batched HNSW search -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never does, and the two share no
code: the only common dependency is the seeded input generator module
``synth``, which holds none of the method's arithmetic.

``oracle.cpp`` (compiled to ``liboracle.so`` by :func:`build`) holds the
arithmetic; this module marshals numpy arrays.  See the header of
``oracle.cpp`` for the paper passages each part follows and for the EXACT and
CANON evaluation modes.

Pieces with no independent pin are marked "parity unpinned" where they are
defined.  Everything here is pinned by the CPU tests (``tests/test_oracle_*``)
against brute force, closed forms, numpy/torch routines or an independent
pure-Python search.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.cpp")

MODES = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3, "pq": 4, "sparse": 5}
METRICS = {"l2": 0, "ip": 1}
KEYS = {"canon": 0, "exact": 1}

CXX_FLAGS = ["-O2", "-std=c++17", "-fopenmp", "-mavx2", "-mfma", "-ffp-contract=off",
             "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so (g++)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", *CXX_FLAGS, SRC_PATH, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int


class OrStore(C.Structure):
    _fields_ = [("mode", C.c_int32), ("metric", C.c_int32), ("d", C.c_int32), ("pad", C.c_int32),
                ("f32", P), ("f16", P), ("fp8", P), ("fp8_scale", P),
                ("pq_m", C.c_int32), ("pq_ksub", C.c_int32), ("pq_dsub", C.c_int32),
                ("pad2", C.c_int32),
                ("pq_cb", P), ("pq_codes", P),
                ("sp_ptr", P), ("sp_ids", P), ("sp_vals", P)]


class OrGraphIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("M", C.c_int32), ("M0", C.c_int32),
                ("max_level", C.c_int32), ("entry", C.c_int32),
                ("levels", P), ("adj0", P), ("upper_off", P), ("upper_adj", P)]


def _declare(L):
    L.or_version.restype = I32
    for f in ("or_to_f16", "or_from_f16", "or_to_bf16", "or_from_bf16", "or_to_e4m3",
              "or_from_e4m3"):
        getattr(L, f).argtypes = [P, I64, P]
        getattr(L, f).restype = None
    L.or_encode_fp8_rows.argtypes = [P, I64, I32, P, P, I32]
    L.or_keys_dense.argtypes = [P, P, I64, P, I64, I32, P, I32]
    L.or_keys_sparse.argtypes = [P, P, P, P, I64, P, I64, I32, P, I32]
    L.or_pq_luts.argtypes = [P, P, I64, I32, P]
    L.or_bruteforce.argtypes = [P, P, P, P, P, I64, I64, I32, I32, P, P, I32]
    L.or_hnsw_build.argtypes = [P, I64, I32, I32, I32, I32, P, I64, C.c_double, I64, I32]
    L.or_hnsw_build.restype = P
    L.or_hnsw_build_sparse.argtypes = [P, P, P, I64, I32, I32, I32, P, I64, C.c_double, I64, I32]
    L.or_hnsw_build_sparse.restype = P
    L.or_graph_info.argtypes = [P, P]
    L.or_graph_export.argtypes = [P, P, P, P, P]
    L.or_graph_free.argtypes = [P]
    L.or_hnsw_search.argtypes = [P, P, P, P, P, P, I64, P, P, I32, I32, P, I32, I32,
                                 P, P, P, P, P, I32, P, I64, I32]
    L.or_pq_train.argtypes = [P, I32, P, I64, P, I32, I32, I32, P, P, I32]
    L.or_pq_train.restype = I32
    L.or_pq_encode.argtypes = [P, I64, I32, P, I32, I32, P, I32]
    L.or_ivf_train.argtypes = [P, I32, P, I64, P, I32, I32, P, P, I32]
    L.or_ivf_train.restype = I32
    L.or_ivf_assign.argtypes = [P, I64, I32, P, I32, P, I32]
    L.or_ivf_search.argtypes = [P, P, I64, P, I32, P, P, I32, I32, I32, P, I32, I32, P, P, P, P,
                                P, P, I32, I32]
    for f in ("or_encode_fp8_rows", "or_keys_dense", "or_keys_sparse", "or_pq_luts",
              "or_bruteforce", "or_graph_info", "or_graph_export", "or_graph_free",
              "or_hnsw_search", "or_pq_encode", "or_ivf_assign", "or_ivf_search"):
        getattr(L, f).restype = None


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def nthreads(threads=None):
    return int(threads or os.cpu_count() or 1)


# --------------------------------------------------------------------------
# Number formats
# --------------------------------------------------------------------------

def to_f16(x):
    x = _c(x, np.float32); out = np.empty(x.shape, np.uint16)
    lib().or_to_f16(_ptr(x), x.size, _ptr(out)); return out


def from_f16(h):
    h = _c(h, np.uint16); out = np.empty(h.shape, np.float32)
    lib().or_from_f16(_ptr(h), h.size, _ptr(out)); return out


def to_bf16(x):
    x = _c(x, np.float32); out = np.empty(x.shape, np.uint16)
    lib().or_to_bf16(_ptr(x), x.size, _ptr(out)); return out


def from_bf16(h):
    h = _c(h, np.uint16); out = np.empty(h.shape, np.float32)
    lib().or_from_bf16(_ptr(h), h.size, _ptr(out)); return out


def to_e4m3(x):
    x = _c(x, np.float32); out = np.empty(x.shape, np.uint8)
    lib().or_to_e4m3(_ptr(x), x.size, _ptr(out)); return out


def from_e4m3(b):
    b = _c(b, np.uint8); out = np.empty(b.shape, np.float32)
    lib().or_from_e4m3(_ptr(b), b.size, _ptr(out)); return out


def encode_fp8_rows(X, threads=None):
    """Per-row scaled E4M3 copy: (codes u8[n,d], scale f32[n])."""
    X = _c(X, np.float32); n, d = X.shape
    codes = np.empty((n, d), np.uint8); scale = np.empty(n, np.float32)
    lib().or_encode_fp8_rows(_ptr(X), n, d, _ptr(codes), _ptr(scale), nthreads(threads))
    return codes, scale


# --------------------------------------------------------------------------
# Stores: what a search reads for each representation
# --------------------------------------------------------------------------

class Store:
    """Arrays of one searchable representation, kept alive with the struct."""

    def __init__(self, mode, metric, d, **arrays):
        self.mode, self.metric, self.d = mode, metric, d
        self.arrays = {k: v for k, v in arrays.items() if v is not None}
        s = OrStore()
        s.mode, s.metric, s.d = MODES[mode], METRICS[metric], d
        a = self.arrays
        s.f32 = _ptr(a.get("f32")); s.fp8 = _ptr(a.get("fp8")); s.fp8_scale = _ptr(a.get("fp8_scale"))
        s.f16 = _ptr(a.get("f16", a.get("bf16")))
        if "pq_cb" in a:
            m, ksub, dsub = a["pq_cb"].shape
            s.pq_m, s.pq_ksub, s.pq_dsub = m, ksub, dsub
            s.pq_cb = _ptr(a["pq_cb"]); s.pq_codes = _ptr(a["pq_codes"])
        s.sp_ptr = _ptr(a.get("sp_ptr")); s.sp_ids = _ptr(a.get("sp_ids")); s.sp_vals = _ptr(a.get("sp_vals"))
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def dense_store(X, metric, mode="f32", fp8_scale=None):
    """X is f32 [n,d] (mode f32), u16 [n,d] (f16/bf16) or u8 [n,d] (fp8)."""
    d = X.shape[1]
    if mode == "f32":
        return Store(mode, metric, d, f32=_c(X, np.float32))
    if mode == "f16":
        return Store(mode, metric, d, f16=_c(X, np.uint16))
    if mode == "bf16":
        return Store(mode, metric, d, bf16=_c(X, np.uint16))
    if mode == "fp8":
        return Store(mode, metric, d, fp8=_c(X, np.uint8), fp8_scale=_c(fp8_scale, np.float32))
    raise ValueError(mode)


def pq_store(codebook, codes, metric):
    codebook = _c(codebook, np.float32)
    m, ksub, dsub = codebook.shape
    return Store("pq", metric, m * dsub, pq_cb=codebook, pq_codes=_c(codes, np.uint8))


def sparse_store(indptr, ids, vals, vocab):
    return Store("sparse", "ip", vocab, sp_ptr=_c(indptr, np.int64), sp_ids=_c(ids, np.uint16),
                 sp_vals=_c(vals, np.float32))


# --------------------------------------------------------------------------
# Keys, brute force
# --------------------------------------------------------------------------

def keys(store, Q, rows, kmode="canon", threads=None, sparse_q=None):
    """keys[i, j] = key(query i, row rows[i, j])."""
    rows = _c(np.atleast_2d(rows), np.int64)
    nq, per = rows.shape
    out = np.empty((nq, per), np.float32)
    if store.mode == "sparse":
        qp, qi, qv = (_c(sparse_q[0], np.int64), _c(sparse_q[1], np.uint16), _c(sparse_q[2], np.float32))
        lib().or_keys_sparse(store.ref, _ptr(qp), _ptr(qi), _ptr(qv), nq, _ptr(rows), per,
                             KEYS[kmode], _ptr(out), nthreads(threads))
    else:
        Q = _c(np.atleast_2d(Q), np.float32)
        lib().or_keys_dense(store.ref, _ptr(Q), nq, _ptr(rows), per, KEYS[kmode], _ptr(out),
                            nthreads(threads))
    return out


def pq_luts(store, Q, kmode="canon"):
    Q = _c(np.atleast_2d(Q), np.float32)
    cb = store.arrays["pq_cb"]
    out = np.empty((Q.shape[0], cb.shape[0], cb.shape[1]), np.float32)
    lib().or_pq_luts(store.ref, _ptr(Q), Q.shape[0], KEYS[kmode], _ptr(out))
    return out


def bruteforce(store, n, k, Q=None, sparse_q=None, kmode="exact", threads=None):
    """Exact k-NN by a full scan, order (key, id).  Returns (ids i64, keys f32)."""
    if store.mode == "sparse":
        qp, qi, qv = (_c(sparse_q[0], np.int64), _c(sparse_q[1], np.uint16), _c(sparse_q[2], np.float32))
        nq = qp.size - 1
        Qp = None
    else:
        Qp = _c(np.atleast_2d(Q), np.float32); nq = Qp.shape[0]
        qp = qi = qv = None
    ids = np.empty((nq, k), np.int64); ks = np.empty((nq, k), np.float32)
    lib().or_bruteforce(store.ref, _ptr(Qp), _ptr(qp), _ptr(qi), _ptr(qv), nq, n, k,
                        KEYS[kmode], _ptr(ids), _ptr(ks), nthreads(threads))
    return ids, ks


# --------------------------------------------------------------------------
# HNSW
# --------------------------------------------------------------------------

class Graph:
    """HNSW graph in the exchange layout (see oracle.cpp)."""

    def __init__(self, n, M, M0, max_level, entry, levels, adj0, upper_off, upper_adj):
        self.n, self.M, self.M0 = int(n), int(M), int(M0)
        self.max_level, self.entry = int(max_level), int(entry)
        self.levels = _c(levels, np.uint8)
        self.adj0 = _c(adj0, np.int32).reshape(self.n, self.M0)
        self.upper_off = _c(upper_off, np.int32)
        self.upper_adj = _c(upper_adj, np.int32).reshape(-1, self.M)

    def struct(self):
        g = OrGraphIn()
        g.n, g.M, g.M0, g.max_level, g.entry = self.n, self.M, self.M0, self.max_level, self.entry
        g.levels = _ptr(self.levels); g.adj0 = _ptr(self.adj0)
        g.upper_off = _ptr(self.upper_off); g.upper_adj = _ptr(self.upper_adj)
        return g

    def neighbours(self, v, lc):
        if lc == 0:
            row = self.adj0[v]
        else:
            row = self.upper_adj[self.upper_off[v] + lc - 1]
        return row[row >= 0]

    def save(self, path):
        """Compact file: layer-0 lists as degrees (u8) + ids packed in 3 bytes
        (little endian; n < 2^24) without padding; upper lists as stored."""
        assert self.n < (1 << 24)
        deg = (self.adj0 >= 0).sum(1).astype(np.uint8)
        ids = self.adj0[self.adj0 >= 0].astype(np.uint32)      # row-major: valid first in each row
        packed = np.stack([(ids >> (8 * b)) & 0xFF for b in range(3)], axis=1).astype(np.uint8)
        np.savez(path, meta=np.array([self.n, self.M, self.M0, self.max_level, self.entry], np.int64),
                 levels=self.levels, deg0=deg, ids0=packed.reshape(-1), upper_off=self.upper_off,
                 upper_adj=self.upper_adj)

    @classmethod
    def load(cls, path):
        z = np.load(path)
        n, M, M0, L, e = (int(v) for v in z["meta"])
        if "adj0" in z:
            adj0 = z["adj0"]
        else:
            deg = z["deg0"].astype(np.int64)
            b = z["ids0"].reshape(-1, 3).astype(np.int32)
            ids = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16)
            adj0 = np.full((n, M0), -1, np.int32)
            adj0[np.arange(M0)[None, :] < deg[:, None]] = ids
        return cls(n, M, M0, L, e, z["levels"], adj0, z["upper_off"], z["upper_adj"])


def hnsw_build(X, metric, M, efc, u_levels, seq_prefix=None, batch_frac=0.0, batch_cap=4096,
               threads=None):
    """Build on FP32 originals.  batch_frac=0 gives purely sequential insertion."""
    X = _c(X, np.float32); n, d = X.shape
    u = _c(u_levels, np.float64)
    assert u.shape == (n,)
    if seq_prefix is None:
        seq_prefix = n
    g = lib().or_hnsw_build(_ptr(X), n, d, METRICS[metric], M, efc, _ptr(u), int(seq_prefix),
                            float(batch_frac), int(batch_cap), nthreads(threads))
    return _export(g, n)


def hnsw_build_sparse(indptr, ids, vals, vocab, M, efc, u_levels, seq_prefix=None,
                      batch_frac=0.0, batch_cap=4096, threads=None):
    """Build over sparse rows (inner product, EXACT merge-join keys)."""
    ip = _c(indptr, np.int64); ii = _c(ids, np.uint16); vv = _c(vals, np.float32)
    n = ip.size - 1
    u = _c(u_levels, np.float64)
    assert u.shape == (n,)
    if seq_prefix is None:
        seq_prefix = n
    g = lib().or_hnsw_build_sparse(_ptr(ip), _ptr(ii), _ptr(vv), n, int(vocab), M, efc, _ptr(u),
                                   int(seq_prefix), float(batch_frac), int(batch_cap),
                                   nthreads(threads))
    return _export(g, n)


def _export(g, n):
    L = lib()
    info = np.zeros(6, np.int64)
    L.or_graph_info(g, _ptr(info))
    n_, M_, M0, max_level, entry, nlists = (int(v) for v in info)
    levels = np.empty(n, np.uint8); adj0 = np.empty((n, M0), np.int32)
    uoff = np.empty(n, np.int32); uadj = np.empty((nlists, M_), np.int32)
    L.or_graph_export(g, _ptr(levels), _ptr(adj0), _ptr(uoff), _ptr(uadj))
    L.or_graph_free(g)
    return Graph(n, M_, M0, max_level, entry, levels, adj0, uoff, uadj)


def hnsw_search(graph, store, k, ef, Q=None, sparse_q=None, kmode="canon", rerank_f32=None,
                rerank=0, rerank_kmode="canon", want_w=False, visited_cap=0, threads=None):
    """HNSW search (Algorithms 5 and 2) with per-query k and ef (scalars or arrays).

    Returns a dict: ids i64[nq,kmax], keys f32[nq,kmax], stats i64[nq,5]
    (evaluations, layer-0 evaluations, layer-0 expansions, |layer-0 visited|,
    |W|), and optionally w_ids/w_keys (W_final sorted) and visited (sorted).
    """
    if store.mode == "sparse":
        qp, qi, qv = (_c(sparse_q[0], np.int64), _c(sparse_q[1], np.uint16), _c(sparse_q[2], np.float32))
        nq = qp.size - 1; Qp = None
    else:
        Qp = _c(np.atleast_2d(Q), np.float32); nq = Qp.shape[0]; qp = qi = qv = None
    k_arr = _c(np.broadcast_to(np.asarray(k), (nq,)), np.int32)
    ef_arr = _c(np.broadcast_to(np.asarray(ef), (nq,)), np.int32)
    kmax = int(k_arr.max()) if nq else 1
    ids = np.empty((nq, kmax), np.int64); ks = np.empty((nq, kmax), np.float32)
    stats = np.empty((nq, 5), np.int64)
    wcap = int(np.maximum(ef_arr, k_arr).max()) if (want_w and nq) else 0
    w_ids = np.empty((nq, wcap), np.int32) if want_w else None
    w_keys = np.empty((nq, wcap), np.float32) if want_w else None
    vis = np.empty((nq, visited_cap), np.int32) if visited_cap else None
    rr = _c(rerank_f32, np.float32)
    g = graph.struct()
    lib().or_hnsw_search(C.byref(g), store.ref, _ptr(Qp), _ptr(qp), _ptr(qi), _ptr(qv), nq,
                         _ptr(k_arr), _ptr(ef_arr), kmax, KEYS[kmode], _ptr(rr), int(rerank),
                         KEYS[rerank_kmode], _ptr(ids), _ptr(ks), _ptr(stats), _ptr(w_ids),
                         _ptr(w_keys), wcap, _ptr(vis), int(visited_cap), nthreads(threads))
    out = dict(ids=ids, keys=ks, stats=stats)
    if want_w:
        out["w_ids"], out["w_keys"] = w_ids, w_keys
    if visited_cap:
        out["visited"] = vis
    return out


# --------------------------------------------------------------------------
# PQ
# --------------------------------------------------------------------------

def pq_train(X, m, ksub, sample_ids, init, max_iter=25, threads=None):
    """k-means per contiguous subspace.  Returns (codebook f32[m,ksub,dsub], iters, objective)."""
    X = _c(X, np.float32); n, d = X.shape
    assert d % m == 0
    s = _c(sample_ids, np.int64); ini = _c(init, np.int64)
    assert ini.size == ksub and ini.max() < s.size
    cb = np.empty((m, ksub, d // m), np.float32)
    obj = np.zeros(max_iter, np.float64)
    it = lib().or_pq_train(_ptr(X), d, _ptr(s), s.size, _ptr(ini), m, ksub, max_iter, _ptr(cb),
                           _ptr(obj), nthreads(threads))
    return cb, int(it), obj


def pq_encode(X, codebook, threads=None):
    X = _c(X, np.float32); n, d = X.shape
    cb = _c(codebook, np.float32); m, ksub, _ = cb.shape
    codes = np.empty((n, m), np.uint8)
    lib().or_pq_encode(_ptr(X), n, d, _ptr(cb), m, ksub, _ptr(codes), nthreads(threads))
    return codes


# --------------------------------------------------------------------------
# IVF (inverted lists over a k-means coarse quantizer)
# --------------------------------------------------------------------------

def ivf_train(X, nlist, sample_ids, init, max_iter=25, threads=None):
    """k-means over whole rows of X[sample_ids].  Returns (centroids f32[nlist,d], iters, objective)."""
    X = _c(X, np.float32); n, d = X.shape
    s = _c(sample_ids, np.int64); ini = _c(init, np.int64)
    assert ini.size == nlist and ini.max() < s.size
    cent = np.empty((nlist, d), np.float32)
    obj = np.zeros(max_iter, np.float64)
    it = lib().or_ivf_train(_ptr(X), d, _ptr(s), s.size, _ptr(ini), nlist, max_iter, _ptr(cent),
                            _ptr(obj), nthreads(threads))
    return cent, int(it), obj


def ivf_assign(X, centroids, threads=None):
    """list[r] = EXACT nearest centroid of row r (lower index on ties), i32[n]."""
    X = _c(X, np.float32); n, d = X.shape
    cent = _c(centroids, np.float32)
    out = np.empty(n, np.int32)
    lib().or_ivf_assign(_ptr(X), n, d, _ptr(cent), cent.shape[0], _ptr(out), nthreads(threads))
    return out


def ivf_lists(assign, nlist):
    """Inverted lists from an assignment: (list_off i64[nlist+1], list_ids i32[n]), ids ascending."""
    a = np.asarray(assign, np.int64)
    order = np.argsort(a, kind="stable").astype(np.int32)
    off = np.zeros(nlist + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(a, minlength=nlist))
    return off, order


def ivf_search(store, centroids, list_off, list_ids, Q, k, nprobe, kmode="canon",
               rerank_f32=None, rerank_depth=0, rerank_kmode="canon", w_cap=0, threads=None):
    """IVF search (see or_ivf_search).  Returns dict(ids, keys, probes, stats[, w_ids, w_keys])."""
    Q = _c(np.atleast_2d(Q), np.float32); nq = Q.shape[0]
    cent = _c(centroids, np.float32); nlist = cent.shape[0]
    off = _c(list_off, np.int64); lid = _c(list_ids, np.int32)
    rr = _c(rerank_f32, np.float32) if rerank_f32 is not None else None
    ids = np.empty((nq, k), np.int64); ks = np.empty((nq, k), np.float32)
    probes = np.empty((nq, nprobe), np.int32); stats = np.empty((nq, 2), np.int64)
    w_ids = np.empty((nq, w_cap), np.int32) if w_cap else None
    w_keys = np.empty((nq, w_cap), np.float32) if w_cap else None
    lib().or_ivf_search(store.ref, _ptr(Q), nq, _ptr(cent), nlist, _ptr(off), _ptr(lid), nprobe, k,
                        KEYS[kmode], _ptr(rr), int(rerank_depth), KEYS[rerank_kmode], _ptr(ids),
                        _ptr(ks), _ptr(probes), _ptr(stats), _ptr(w_ids), _ptr(w_keys), int(w_cap),
                        nthreads(threads))
    out = dict(ids=ids, keys=ks, probes=probes, stats=stats)
    if w_cap:
        out["w_ids"], out["w_keys"] = w_ids, w_keys
    return out


# --------------------------------------------------------------------------
# Recall
# --------------------------------------------------------------------------

def recall_at_k(found_ids, gt_ids, k):
    """Mean over queries of |found[:k] & gt[:k]| / k."""
    found = np.asarray(found_ids)[:, :k]; gt = np.asarray(gt_ids)[:, :k]
    hits = [len(set(f[f >= 0].tolist()) & set(g.tolist())) for f, g in zip(found, gt)]
    return float(np.mean(hits)) / k if len(hits) else 0.0
