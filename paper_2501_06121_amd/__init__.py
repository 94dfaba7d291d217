"""Python binding of libann.so, the MI355X batched HNSW search library.

Argument marshalling only: every step of a search runs in the library's HIP
kernels (see include/ann.h for the operations and their conventions).  Torch
is used for device memory and streams.  The functions carry the names of the
C entry points.

The library must have been built (``python -m paper_2501_06121_amd.build``);
importing a function that needs it raises if ``libann.so`` is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libann.so")

ANN_OK, ANN_EINVAL, ANN_ENODEV, ANN_ENOMEM, ANN_EBUDGET, ANN_EFORMAT, ANN_EHIP, ANN_EUNSUP, \
    ANN_EAGAIN = range(9)
ERR_NAMES = {0: "ANN_OK", 1: "ANN_EINVAL", 2: "ANN_ENODEV", 3: "ANN_ENOMEM", 4: "ANN_EBUDGET",
             5: "ANN_EFORMAT", 6: "ANN_EHIP", 7: "ANN_EUNSUP", 8: "ANN_EAGAIN"}
METRIC = {"l2": 0, "ip": 1}
MODE = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3, "pq": 4, "sparse": 5}
ANN_EF_MAX = 65536
ANN_BEAM_AUTO, ANN_BEAM_LDS, ANN_BEAM_HBM = 0, 1, 2
ANN_K_MAX = 1024

P = C.c_void_p
I32, I64, U64, F64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double


class AnnIndexDesc(C.Structure):
    _fields_ = [("n", I64), ("d", I32), ("metric", I32), ("M", I32), ("M0", I32),
                ("max_level", I32), ("entry_point", I32), ("n_upper_lists", I64),
                ("levels", P), ("adj0", P), ("upper_off", P), ("upper_adj", P),
                ("x_f32", P), ("x_f16", P), ("x_bf16", P), ("x_fp8", P), ("fp8_scale", P),
                ("pq_m", I32), ("pq_ksub", I32), ("pq_codebook", P), ("pq_codes", P),
                ("sp_indptr", P), ("sp_ids", P), ("sp_vals", P)]


class AnnIndexInfo(C.Structure):
    _fields_ = [("n", I64), ("d", I32), ("metric", I32), ("M", I32), ("M0", I32),
                ("max_level", I32), ("entry_point", I32), ("modes", I32), ("device", I32),
                ("device_bytes", I64)]


class AnnBatch(C.Structure):
    _fields_ = [("mode", I32), ("rerank", I32), ("nq", I64),
                ("queries", P), ("q_indptr", P), ("q_ids", P), ("q_vals", P),
                ("k", P), ("ef", P), ("k_all", I32), ("ef_all", I32), ("k_max", I32),
                ("ef_max", I32), ("out_ids", P), ("out_dists", P), ("out_status", P),
                ("out_stats", P), ("out_visited", P), ("visited_cap", I64)]


class AnnLaunchCfg(C.Structure):
    _fields_ = [("slots", I32), ("lanes_per_row", I32), ("waves_per_query", I32),
                ("beam_buffer", I32), ("beam_list", I32)]


class AnnServerCfg(C.Structure):
    _fields_ = [("mode", I32), ("rerank", I32), ("max_inflight", I32), ("slots", I32),
                ("k_max", I32), ("ef_max", I32), ("queue_cap", I32), ("idle_us", I32),
                ("hbm_budget", I64)]


class AnnServerState(C.Structure):
    _fields_ = [("slots", I32), ("ring", I32), ("waves_per_query", I32), ("lanes_per_row", I32),
                ("queued", I64)]


class AnnRequest(C.Structure):
    _fields_ = [("tag", U64), ("query", P), ("k", I32), ("ef", I32)]


class AnnCompletion(C.Structure):
    _fields_ = [("tag", U64), ("status", I32), ("k", I32), ("ids", I64 * ANN_K_MAX),
                ("dists", C.c_float * ANN_K_MAX), ("t_submit", F64), ("t_start", F64),
                ("t_done", F64), ("d_start", F64), ("d_done", F64), ("slot", I32),
                ("reserved", I32)]


# Every exported symbol and its argument types; the CPU tests check that the
# library exports all of them.
class AnnIvfBatch(C.Structure):
    _fields_ = [("mode", I32), ("rerank", I32), ("nq", I64), ("queries", P), ("k", I32),
                ("nprobe", I32), ("out_ids", P), ("out_dists", P), ("out_probes", P),
                ("out_stats", P), ("group", I32)]


SIGNATURES = {
    "ann_index_create": ([P, C.c_int, P], C.c_int),
    "ann_index_free": ([P], C.c_int),
    "ann_index_info": ([P, P], C.c_int),
    "ann_index_info_get": ([P, P], C.c_int),
    "ann_index_file_info": ([C.c_char_p, P], C.c_int),
    "ann_index_load": ([C.c_char_p, C.c_int, P], C.c_int),
    "ann_index_save": ([P, C.c_char_p], C.c_int),
    "ann_search": ([P, P, I64, I32, I32, P, P], C.c_int),
    "ann_search_ex": ([P, P, P], C.c_int),
    "ann_search_sparse": ([P, P, P, P, I64, I32, I32, P, P], C.c_int),
    "ann_set_launch": ([P, I32, P], C.c_int),
    "ann_get_launch": ([P, I32, P], C.c_int),
    "ann_autotune": ([P, P, P], C.c_int),
    "ann_plan_create": ([P, P, P, P], C.c_int),
    "ann_plan_launch": ([P, P], C.c_int),
    "ann_plan_info": ([P, P], C.c_int),
    "ann_plan_free": ([P], C.c_int),
    "ann_bruteforce": ([P, P, I64, I32, P, P, P, P], C.c_int),
    "ann_bruteforce_noalloc": ([P, P, I64, I32, P, P, P, P], C.c_int),
    "ann_pq_train": ([P, I64, I32, P, I64, P, I32, I32, I32, P, P, P], C.c_int),
    "ann_pq_encode": ([P, I64, I32, P, I32, I32, P, P], C.c_int),
    "ann_hnsw_build": ([P, I64, I32, I32, I32, I32, P, I64, C.c_double, I64, P, P], C.c_int),
    "ann_graph_info": ([P, P], C.c_int),
    "ann_graph_export": ([P, P, P, P, P], C.c_int),
    "ann_graph_free": ([P], C.c_int),
    "ann_encode_fp8": ([P, I64, I32, P, P, P], C.c_int),
    "ann_ivf_train": ([P, I64, I32, P, I64, P, I32, I32, P, P, P], C.c_int),
    "ann_ivf_assign": ([P, I64, I32, P, I32, P, P], C.c_int),
    "ann_ivf_group": ([P, I64, I32, P, P], C.c_int),
    "ann_ivf_create": ([P, I32, P, P, P, P], C.c_int),
    "ann_ivf_free": ([P], C.c_int),
    "ann_ivf_search": ([P, P, P], C.c_int),
    "ann_server_create": ([P, P, P], C.c_int),
    "ann_server_submit": ([P, P], C.c_int),
    "ann_server_poll": ([P, P, I32], C.c_int),
    "ann_server_info": ([P, P], C.c_int),
    "ann_server_destroy": ([P], C.c_int),
    "ann_last_error": ([], C.c_char_p),
    "ann_version": ([], C.c_int),
    "ann_debug_flags": ([P, C.POINTER(C.c_uint32), C.c_int32], C.c_int),
    "ann_device_count": ([], C.c_int),
}

_lib = None


def _load_hip_runtime():
    """Load the HIP runtime PyTorch uses before the library.

    The library was linked against that runtime; loading it first makes the
    library bind to the same copy (matched by its soname), so that torch and
    the library share one runtime and one view of the GPU.
    """
    try:
        import torch
    except ImportError:
        return
    rt = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    if os.path.exists(rt):
        C.CDLL(rt, mode=getattr(os, "RTLD_GLOBAL", 0x100))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2501_06121_amd.build` (no fallback exists)")
        _load_hip_runtime()
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class AnnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != ANN_OK:
        raise AnnError(rc, lib().ann_last_error().decode())
    return rc


def _np(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _hptr(a):
    return None if a is None else a.ctypes.data


def _dptr(t):
    return None if t is None else t.data_ptr()


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# --------------------------------------------------------------------------
# index
# --------------------------------------------------------------------------

class Index:
    """Owns an ann_index handle; freed with ann_index_free on close/GC."""

    def __init__(self, handle, d, metric):
        self.handle = handle
        self.d = d
        self.metric = metric

    def close(self):
        if self.handle:
            lib().ann_index_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = AnnIndexInfo()
        _check(lib().ann_index_info(self.handle, C.byref(out)))
        return {f: getattr(out, f) for f, _ in AnnIndexInfo._fields_}


def _desc(graph, metric, d, x_f32=None, x_f16=None, x_bf16=None, x_fp8=None, fp8_scale=None,
          pq_codebook=None, pq_codes=None, sp_indptr=None, sp_ids=None, sp_vals=None):
    """An AnnIndexDesc over host arrays, and the arrays it points into."""
    keep = dict(levels=_np(graph.levels, np.uint8), adj0=_np(graph.adj0, np.int32),
                upper_off=_np(graph.upper_off, np.int32), upper_adj=_np(graph.upper_adj, np.int32),
                x_f32=_np(x_f32, np.float32), x_f16=_np(x_f16, np.uint16),
                x_bf16=_np(x_bf16, np.uint16), x_fp8=_np(x_fp8, np.uint8),
                fp8_scale=_np(fp8_scale, np.float32), pq_codebook=_np(pq_codebook, np.float32),
                pq_codes=_np(pq_codes, np.uint8), sp_indptr=_np(sp_indptr, np.int64),
                sp_ids=_np(sp_ids, np.uint16), sp_vals=_np(sp_vals, np.float32))
    D = AnnIndexDesc()
    D.n, D.d, D.metric = int(graph.n), int(d), METRIC[metric]
    D.M, D.M0, D.max_level, D.entry_point = int(graph.M), int(graph.M0), int(graph.max_level), int(graph.entry)
    D.n_upper_lists = int(keep["upper_adj"].size // max(1, int(graph.M)))
    for k, v in keep.items():
        setattr(D, k, _hptr(v))
    if keep["pq_codes"] is not None:
        D.pq_m = int(keep["pq_codes"].shape[1])
        D.pq_ksub = int(keep["pq_codebook"].shape[1])
    return D, keep


def ann_index_create(graph, metric, d, device=0, **arrays):
    """Copy host arrays to the device.  `graph` has the attributes n, M, M0,
    max_level, entry, levels, adj0, upper_off, upper_adj (exchange layout);
    `arrays` are x_f32, x_f16, x_bf16, x_fp8, fp8_scale, pq_codebook,
    pq_codes, sp_indptr, sp_ids, sp_vals (the ann_index_desc fields)."""
    D, keep = _desc(graph, metric, d, **arrays)
    h = P()
    _check(lib().ann_index_create(C.byref(D), int(device), C.byref(h)))
    return Index(h, int(d), metric)


def ann_index_save(path, graph, metric, d, **arrays):
    """Write the host arrays of an index to an index file (host only)."""
    D, keep = _desc(graph, metric, d, **arrays)
    _check(lib().ann_index_save(C.byref(D), os.fsencode(path)))


def ann_index_file_info(path):
    """Check an index file on the host (no GPU) and describe it."""
    out = AnnIndexInfo()
    _check(lib().ann_index_file_info(os.fsencode(path), C.byref(out)))
    return {f: getattr(out, f) for f, _ in AnnIndexInfo._fields_}


def ann_index_load(path, device=0):
    """Check an index file and copy its arrays to GPU `device`."""
    info = ann_index_file_info(path)
    h = P()
    _check(lib().ann_index_load(os.fsencode(path), int(device), C.byref(h)))
    return Index(h, int(info["d"]), "ip" if info["metric"] == METRIC["ip"] else "l2")


def ann_index_free(index):
    index.close()


# --------------------------------------------------------------------------
# search
# --------------------------------------------------------------------------

def ann_search(index, queries, k, ef):
    """FP32 search, one k and ef; queries: cuda float32 [nq, d].  Blocking."""
    torch = _torch()
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
    dists = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    _check(lib().ann_search(index.handle, _dptr(queries), nq, int(k), int(ef), _dptr(ids),
                            _dptr(dists)))
    return ids, dists


def ann_search_ex(index, mode="f32", queries=None, sparse=None, k=10, ef=64, rerank=0,
                  k_max=None, ef_max=None, stream=None, want_stats=False, visited_cap=0,
                  out=None):
    """Batched search with per-query k/ef (ints or cuda int32 tensors).

    sparse = (indptr i64, ids i16/i32->u16, vals f32) cuda tensors.  With
    stream=None the call runs on the index stream and blocks; with a torch
    stream it is asynchronous on that stream.  Returns a dict of tensors.
    """
    torch = _torch()
    if sparse is not None:
        q_ptr, q_ids, q_vals = sparse
        nq = q_ptr.shape[0] - 1
        dev = q_ptr.device
    else:
        nq = queries.shape[0]
        dev = queries.device
    b = AnnBatch()
    b.mode = MODE[mode] if isinstance(mode, str) else int(mode)
    b.rerank = int(rerank)
    b.nq = nq
    b.queries = _dptr(queries)
    if sparse is not None:
        b.q_indptr, b.q_ids, b.q_vals = _dptr(q_ptr), _dptr(q_ids), _dptr(q_vals)
    if torch.is_tensor(k):
        b.k = _dptr(k)
        b.k_max = int(k_max if k_max is not None else int(k.max().item()) if nq else 1)
    else:
        b.k_all = int(k)
        b.k_max = int(k_max if k_max is not None else k)
    if torch.is_tensor(ef):
        b.ef = _dptr(ef)
        b.ef_max = int(ef_max if ef_max is not None else int(ef.max().item()) if nq else 1)
    else:
        b.ef_all = int(ef)
        b.ef_max = int(ef_max if ef_max is not None else ef)
    res = out or {}
    if "ids" not in res:
        res["ids"] = torch.empty((nq, b.k_max), dtype=torch.int64, device=dev)
        res["dists"] = torch.empty((nq, b.k_max), dtype=torch.float32, device=dev)
        res["status"] = torch.empty((nq,), dtype=torch.int32, device=dev)
        if want_stats:
            res["stats"] = torch.empty((nq, 4), dtype=torch.int32, device=dev)
        if visited_cap:
            res["visited"] = torch.empty((nq, visited_cap), dtype=torch.int32, device=dev)
    b.out_ids, b.out_dists = _dptr(res["ids"]), _dptr(res["dists"])
    b.out_status = _dptr(res.get("status"))
    b.out_stats = _dptr(res.get("stats"))
    if "visited" in res:
        b.out_visited = _dptr(res["visited"])
        b.visited_cap = res["visited"].shape[1]
    _check(lib().ann_search_ex(index.handle, C.byref(b), _stream_handle(stream)))
    return res


def ann_search_sparse(index, indptr, ids, vals, k, ef):
    torch = _torch()
    nq = indptr.shape[0] - 1
    out_ids = torch.empty((nq, k), dtype=torch.int64, device=indptr.device)
    out_d = torch.empty((nq, k), dtype=torch.float32, device=indptr.device)
    _check(lib().ann_search_sparse(index.handle, _dptr(indptr), _dptr(ids), _dptr(vals), nq,
                                   int(k), int(ef), _dptr(out_ids), _dptr(out_d)))
    return out_ids, out_d


BEAM_LIST = {"auto": ANN_BEAM_AUTO, "lds": ANN_BEAM_LDS, "hbm": ANN_BEAM_HBM}


def ann_set_launch(index, mode, slots=0, lanes_per_row=0, waves_per_query=0, beam_buffer=0,
                   beam_list="auto"):
    bl = BEAM_LIST[beam_list] if isinstance(beam_list, str) else int(beam_list)
    cfg = AnnLaunchCfg(int(slots), int(lanes_per_row), int(waves_per_query), int(beam_buffer), bl)
    _check(lib().ann_set_launch(index.handle, MODE[mode] if isinstance(mode, str) else int(mode),
                                C.byref(cfg)))


def ann_get_launch(index, mode):
    cfg = AnnLaunchCfg()
    _check(lib().ann_get_launch(index.handle, MODE[mode] if isinstance(mode, str) else int(mode),
                                C.byref(cfg)))
    return {"slots": cfg.slots, "lanes_per_row": cfg.lanes_per_row,
            "waves_per_query": cfg.waves_per_query, "beam_buffer": cfg.beam_buffer,
            "beam_list": cfg.beam_list}


def ann_autotune(index, mode="f32", queries=None, sparse=None, k=10, ef=64, rerank=0):
    torch = _torch()
    nq = queries.shape[0] if queries is not None else sparse[0].shape[0] - 1
    dev = queries.device if queries is not None else sparse[0].device
    ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    b = AnnBatch()
    b.mode = MODE[mode]
    b.rerank = int(rerank)
    b.nq = nq
    b.queries = _dptr(queries)
    if sparse is not None:
        b.q_indptr, b.q_ids, b.q_vals = (_dptr(t) for t in sparse)
    b.k_all, b.k_max, b.ef_all, b.ef_max = int(k), int(k), int(ef), int(max(ef, k))
    b.out_ids, b.out_dists = _dptr(ids), _dptr(dists)
    cfg = AnnLaunchCfg()
    _check(lib().ann_autotune(index.handle, C.byref(b), C.byref(cfg)))
    return {"slots": cfg.slots, "lanes_per_row": cfg.lanes_per_row,
            "waves_per_query": cfg.waves_per_query, "beam_buffer": cfg.beam_buffer,
            "beam_list": cfg.beam_list}


class Plan:
    """A captured batch (ann_plan_*): fixed device buffers for up to
    `capacity` queries; refill ``queries`` (and ``k`` / ``ef`` when per-query)
    in place, then ``launch(nq)`` replays the graph for the first nq."""

    def __init__(self, index, mode, capacity, k=10, ef=64, rerank=0, k_max=None, ef_max=None,
                 per_query=False, device="cuda:0"):
        torch = _torch()
        self.index = index
        d = index.d
        self.queries = torch.zeros((capacity, d), dtype=torch.float32, device=device)
        self.nq = torch.zeros((1,), dtype=torch.int32, device=device)
        k_max = int(k_max if k_max is not None else k)
        ef_max = int(ef_max if ef_max is not None else ef)
        self.k = torch.full((capacity,), int(k), dtype=torch.int32, device=device) if per_query else None
        self.ef = torch.full((capacity,), int(ef), dtype=torch.int32, device=device) if per_query else None
        self.ids = torch.empty((capacity, k_max), dtype=torch.int64, device=device)
        self.dists = torch.empty((capacity, k_max), dtype=torch.float32, device=device)
        self.status = torch.empty((capacity,), dtype=torch.int32, device=device)
        self.stats = torch.empty((capacity, 4), dtype=torch.int32, device=device)
        b = AnnBatch()
        b.mode = MODE[mode] if isinstance(mode, str) else int(mode)
        b.rerank = int(rerank)
        b.nq = int(capacity)
        b.queries = _dptr(self.queries)
        b.k, b.ef = _dptr(self.k), _dptr(self.ef)
        b.k_all, b.ef_all, b.k_max, b.ef_max = int(k), int(ef), k_max, ef_max
        b.out_ids, b.out_dists = _dptr(self.ids), _dptr(self.dists)
        b.out_status, b.out_stats = _dptr(self.status), _dptr(self.stats)
        self.handle = P()
        torch.cuda.synchronize()
        _check(lib().ann_plan_create(index.handle, C.byref(b), _dptr(self.nq), C.byref(self.handle)))

    def launch(self, nq=None, stream=None):
        """Set the batch size on the device (on `stream`) and replay."""
        torch = _torch()
        if nq is not None:
            if stream is None:
                self.nq.fill_(int(nq))
                torch.cuda.current_stream().synchronize()
            else:
                with torch.cuda.stream(stream):
                    self.nq.fill_(int(nq))
        _check(lib().ann_plan_launch(self.handle, _stream_handle(stream)))

    def info(self):
        cfg = AnnLaunchCfg()
        _check(lib().ann_plan_info(self.handle, C.byref(cfg)))
        return {"slots": cfg.slots, "lanes_per_row": cfg.lanes_per_row,
                "waves_per_query": cfg.waves_per_query, "beam_buffer": cfg.beam_buffer,
                "beam_list": cfg.beam_list}

    def close(self):
        if self.handle:
            lib().ann_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ann_bruteforce(index, queries, k, stream=None):
    """Exact k-NN on matrix cores; returns (ids, dists, certified) tensors."""
    torch = _torch()
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
    dists = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    cert = torch.empty((nq,), dtype=torch.int32, device=queries.device)
    _check(lib().ann_bruteforce(index.handle, _dptr(queries), nq, int(k), _dptr(ids), _dptr(dists),
                                _dptr(cert), _stream_handle(stream)))
    return ids, dists, cert


class BuiltGraph:
    """A graph built on the device, in the index layout (host numpy arrays)."""

    def __init__(self, n, M, M0, max_level, entry, levels, adj0, upper_off, upper_adj):
        self.n, self.M, self.M0, self.max_level, self.entry = n, M, M0, max_level, entry
        self.levels, self.adj0, self.upper_off, self.upper_adj = levels, adj0, upper_off, upper_adj


def ann_hnsw_build(X, metric, M, efc, u_levels, seq_prefix=None, batch_frac=0.0, batch_cap=4096,
                   stream=None):
    """HNSW construction on the device over X (device f32[n, d]); u_levels:
    host f64[n].  seq_prefix None means every node is inserted alone."""
    n, d = X.shape
    u = np.ascontiguousarray(u_levels, dtype=np.float64)
    assert u.shape == (n,)
    if seq_prefix is None:
        seq_prefix = n
    g = C.c_void_p()
    _check(lib().ann_hnsw_build(_dptr(X), n, d, METRIC[metric], int(M), int(efc), _hptr(u),
                                int(seq_prefix), float(batch_frac), int(batch_cap), C.byref(g),
                                _stream_handle(stream)))
    try:
        info = np.zeros(6, np.int64)
        _check(lib().ann_graph_info(g, _hptr(info)))
        n_, M_, M0, max_level, entry, nlists = (int(v) for v in info)
        levels = np.empty(n_, np.uint8)
        adj0 = np.empty((n_, M0), np.int32)
        uoff = np.empty(n_, np.int32)
        uadj = np.empty((nlists, M_), np.int32)
        _check(lib().ann_graph_export(g, _hptr(levels), _hptr(adj0), _hptr(uoff), _hptr(uadj)))
    finally:
        lib().ann_graph_free(g)
    return BuiltGraph(n_, M_, M0, max_level, entry, levels, adj0, uoff, uadj)


def ann_pq_train(X, sample, init, m, ksub=256, max_iter=25, stream=None):
    """k-means per subspace on the device.  X: device f32[n, d]; sample, init:
    device i64 (row ids; positions into sample).  Returns (codebook f32[m, ksub,
    d/m] on X's device, iterations run)."""
    torch = _torch()
    n, d = X.shape
    cb = torch.empty((m, ksub, d // m), dtype=torch.float32, device=X.device)
    iters = C.c_int32(0)
    _check(lib().ann_pq_train(_dptr(X), n, d, _dptr(sample), sample.shape[0], _dptr(init), int(m),
                              int(ksub), int(max_iter), _dptr(cb), C.byref(iters),
                              _stream_handle(stream)))
    return cb, iters.value


def ann_pq_encode(X, codebook, stream=None):
    """Codes u8[n, m] of the rows of X (device f32[n, d]) for a device codebook."""
    torch = _torch()
    n, d = X.shape
    m, ksub, _ = codebook.shape
    codes = torch.empty((n, m), dtype=torch.uint8, device=X.device)
    _check(lib().ann_pq_encode(_dptr(X), n, d, _dptr(codebook), int(m), int(ksub), _dptr(codes),
                               _stream_handle(stream)))
    return codes


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

# --------------------------------------------------------------------------
# IVF index
# --------------------------------------------------------------------------

class Ivf:
    """Owns an ann_ivf handle (inverted lists over an Index, which it keeps alive)."""

    def __init__(self, handle, index, nlist):
        self.handle, self.index, self.nlist = handle, index, nlist

    def close(self):
        if self.handle:
            lib().ann_ivf_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ann_encode_fp8(X, stream=None):
    """FP8-E4M3 rows with per-row scales of cuda f32 [n, d]: (codes u8 [n, d], scale f32 [n])."""
    torch = _torch()
    n, d = X.shape
    codes = torch.empty((n, d), dtype=torch.uint8, device=X.device)
    scale = torch.empty((n,), dtype=torch.float32, device=X.device)
    _check(lib().ann_encode_fp8(_dptr(X), n, d, _dptr(codes), _dptr(scale), _stream_handle(stream)))
    return codes, scale


def ann_ivf_train(X, sample, init, nlist, max_iter=25, stream=None):
    """k-means of the coarse quantizer on the device.  X cuda f32 [n, d];
    sample, init cuda i64.  Returns (centroids cuda f32 [nlist, d], iterations)."""
    torch = _torch()
    n, d = X.shape
    cent = torch.empty((nlist, d), dtype=torch.float32, device=X.device)
    it = C.c_int32(0)
    _check(lib().ann_ivf_train(_dptr(X), n, d, _dptr(sample), sample.shape[0], _dptr(init), int(nlist),
                               int(max_iter), _dptr(cent), C.byref(it), _stream_handle(stream)))
    return cent, int(it.value)


def ann_ivf_assign(X, centroids, stream=None):
    """Nearest centroid of every row (cuda i32 [n])."""
    torch = _torch()
    n, d = X.shape
    out = torch.empty((n,), dtype=torch.int32, device=X.device)
    _check(lib().ann_ivf_assign(_dptr(X), n, d, _dptr(centroids), centroids.shape[0], _dptr(out),
                                _stream_handle(stream)))
    return out


def ann_ivf_group(assign, nlist):
    """Host lists of an assignment: (list_off i64[nlist+1], list_ids i32[n])."""
    a = _np(assign, np.int32)
    off = np.empty(nlist + 1, np.int64)
    ids = np.empty(a.size, np.int32)
    _check(lib().ann_ivf_group(_hptr(a), a.size, int(nlist), _hptr(off), _hptr(ids)))
    return off, ids


def ann_ivf_create(index, centroids, list_off, list_ids):
    """Host arrays: centroids f32[nlist, d], list_off i64[nlist+1], list_ids i32[n]."""
    cent = _np(centroids, np.float32)
    off = _np(list_off, np.int64)
    ids = _np(list_ids, np.int32)
    h = P()
    _check(lib().ann_ivf_create(index.handle, int(cent.shape[0]), _hptr(cent), _hptr(off),
                                _hptr(ids), C.byref(h)))
    return Ivf(h, index, int(cent.shape[0]))


def ann_ivf_free(ivf):
    ivf.close()


def ann_ivf_search(ivf, queries, k, nprobe, mode="f32", rerank=0, want_probes=False,
                   want_stats=False, stream=None, out=None, group=0):
    """IVF search of cuda float32 queries [nq, d].  Returns a dict of tensors
    (ids, dists[, probes][, stats]).  Blocking unless a stream is given."""
    torch = _torch()
    nq = queries.shape[0]
    dev = queries.device
    res = out or {}
    if "ids" not in res:
        res["ids"] = torch.empty((nq, k), dtype=torch.int64, device=dev)
        res["dists"] = torch.empty((nq, k), dtype=torch.float32, device=dev)
        if want_probes:
            res["probes"] = torch.empty((nq, nprobe), dtype=torch.int32, device=dev)
        if want_stats:
            res["stats"] = torch.empty((nq, 2), dtype=torch.int32, device=dev)
    b = AnnIvfBatch()
    b.mode = MODE[mode] if isinstance(mode, str) else int(mode)
    b.rerank, b.nq, b.queries = int(rerank), nq, _dptr(queries)
    b.k, b.nprobe = int(k), int(nprobe)
    b.out_ids, b.out_dists = _dptr(res["ids"]), _dptr(res["dists"])
    b.out_probes = _dptr(res.get("probes"))
    b.out_stats = _dptr(res.get("stats"))
    b.group = int(group)
    _check(lib().ann_ivf_search(ivf.handle, C.byref(b), _stream_handle(stream)))
    return res


class Server:
    """Continuous batching with per-slot admission around ann_server_* (host
    query vectors in, completions out)."""

    def __init__(self, index, mode="f16", rerank=0, max_inflight=4096, slots=0, k_max=100,
                 ef_max=512, queue_cap=1 << 16, idle_us=0, hbm_budget=8 << 30):
        cfg = AnnServerCfg(MODE[mode], int(rerank), int(max_inflight), int(slots), int(k_max),
                           int(ef_max), int(queue_cap), int(idle_us), int(hbm_budget))
        self.index = index
        self.handle = P()
        _check(lib().ann_server_create(index.handle, C.byref(cfg), C.byref(self.handle)))
        self._buf = (AnnCompletion * 256)()

    def submit(self, tag, query, k, ef):
        q = np.ascontiguousarray(query, dtype=np.float32)
        r = AnnRequest(int(tag), q.ctypes.data, int(k), int(ef))
        rc = lib().ann_server_submit(self.handle, C.byref(r))
        if rc == ANN_EAGAIN:
            return False
        _check(rc)
        return True

    def poll(self):
        n = lib().ann_server_poll(self.handle, self._buf, len(self._buf))
        if n < 0:
            _check(-n)
        out = []
        for i in range(n):
            c = self._buf[i]
            kk = c.k
            out.append(dict(tag=c.tag, status=c.status, ids=np.array(c.ids[:kk], np.int64),
                            dists=np.array(c.dists[:kk], np.float32), t_submit=c.t_submit,
                            t_start=c.t_start, t_done=c.t_done, d_start=c.d_start,
                            d_done=c.d_done, slot=c.slot))
        return out

    def info(self):
        st = AnnServerState()
        _check(lib().ann_server_info(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in AnnServerState._fields_}

    def close(self):
        if self.handle:
            _check(lib().ann_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ann_version():
    return lib().ann_version()


def ann_debug_flags(index, clear=True):
    """Invariant-violation bits of a library built with ANN_DEBUG_CHECKS
    (libann_debug.so); raises AnnError (ANN_EUNSUP) for the regular one."""
    out = C.c_uint32(0)
    _check(lib().ann_debug_flags(index.handle, C.byref(out), 1 if clear else 0))
    return out.value


def ann_device_count():
    return lib().ann_device_count()
