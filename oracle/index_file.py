"""Index files, written and read by the oracle (test infrastructure).

An independent implementation of the documented version-1 index file (the
layout is specified next to ``ann_index_load`` in the library's C header):
a 128-byte header, a table of sections with one CRC-32 each and the arrays
at 64-byte boundaries, little-endian.  It shares nothing with the library's
reader and writer; the tests check that each side reads what the other
writes, and that both write the same bytes for the same arrays.

Only the tests, the smoke check and the benchmark's CPU baseline use this.
"""
from __future__ import annotations

import struct
import zlib

import numpy as np

MAGIC = b"ANNINDEX"
VERSION = 1
HEADER = 128
ENTRY = 32
ALIGN = 64

# id: (name, dtype)
SECTIONS = {
    1: ("levels", np.uint8), 2: ("adj0", np.int32), 3: ("upper_off", np.int32),
    4: ("upper_adj", np.int32), 5: ("x_f32", np.float32), 6: ("x_f16", np.uint16),
    7: ("x_bf16", np.uint16), 8: ("x_fp8", np.uint8), 9: ("fp8_scale", np.float32),
    10: ("pq_codebook", np.float32), 11: ("pq_codes", np.uint8), 12: ("sp_indptr", np.int64),
    13: ("sp_ids", np.uint16), 14: ("sp_vals", np.float32),
}
NAME_TO_ID = {v[0]: k for k, v in SECTIONS.items()}
METRICS = {"l2": 0, "ip": 1}


def _pad(n):
    return (n + ALIGN - 1) // ALIGN * ALIGN


def _shapes(h):
    """Element shape of every section under the header's fields."""
    n, d, m = h["n"], h["d"], h["pq_m"]
    return {
        "levels": (n,), "adj0": (n, h["M0"]), "upper_off": (n,), "upper_adj": (h["n_upper_lists"], h["M"]),
        "x_f32": (n, d), "x_f16": (n, d), "x_bf16": (n, d), "x_fp8": (n, d), "fp8_scale": (n,),
        "pq_codebook": (m, 256, d // m if m else 0), "pq_codes": (n, m), "sp_indptr": (n + 1,),
        "sp_ids": (h["nnz"],), "sp_vals": (h["nnz"],),
    }


def write(path, graph, metric, d, **arrays):
    """Write the graph (attributes n, M, M0, max_level, entry, levels, adj0,
    upper_off, upper_adj) and the representation arrays named as in the
    library's index description (x_f32, x_f16, ...) to `path`."""
    a = {k: v for k, v in arrays.items() if v is not None}
    a["levels"], a["adj0"], a["upper_off"] = graph.levels, graph.adj0, graph.upper_off
    n_upper = int(np.asarray(graph.upper_adj).size // max(1, int(graph.M)))
    if n_upper:
        a["upper_adj"] = graph.upper_adj
    if "x_fp8" not in a:
        a.pop("fp8_scale", None)
    pq_m = int(np.asarray(a["pq_codes"]).shape[1]) if "pq_codes" in a else 0
    if not pq_m:
        a.pop("pq_codebook", None)
    nnz = int(np.asarray(a["sp_indptr"])[-1]) if "sp_indptr" in a else 0
    if not nnz:
        for k in ("sp_indptr", "sp_ids", "sp_vals"):
            a.pop(k, None)
    ids = sorted(NAME_TO_ID[k] for k in a)
    blobs = {i: np.ascontiguousarray(a[SECTIONS[i][0]], dtype=SECTIONS[i][1]).tobytes() for i in ids}
    head = bytearray(HEADER)
    head[0:8] = MAGIC
    struct.pack_into("<IIqiiiiiiqiiq", head, 8, VERSION, len(ids), int(graph.n), int(d),
                     METRICS[metric], int(graph.M), int(graph.M0), int(graph.max_level),
                     int(graph.entry), n_upper, pq_m, 256 if pq_m else 0, nnz)
    struct.pack_into("<I", head, 124, zlib.crc32(bytes(head[:124])))
    table = bytearray()
    off = _pad(HEADER + ENTRY * len(ids) + 4)
    offsets = []
    for i in ids:
        table += struct.pack("<IIQQQ", i, zlib.crc32(blobs[i]), off, len(blobs[i]), 0)
        offsets.append(off)
        off = _pad(off + len(blobs[i]))
    out = bytearray(head) + table + struct.pack("<I", zlib.crc32(bytes(table)))
    with open(path, "wb") as f:
        f.write(out)
        pos = len(out)
        for i, o in zip(ids, offsets):
            f.write(b"\0" * (o - pos))
            f.write(blobs[i])
            pos = o + len(blobs[i])


def read(path):
    """Parse and check a file; returns (header dict, {name: array}).
    Raises ValueError naming the first problem found."""
    raw = open(path, "rb").read()
    if len(raw) < HEADER:
        raise ValueError("shorter than the header")
    if raw[:8] != MAGIC:
        raise ValueError("magic")
    fields = struct.unpack_from("<IIqiiiiiiqiiq", raw, 8)
    keys = ("version", "sections", "n", "d", "metric", "M", "M0", "max_level", "entry_point",
            "n_upper_lists", "pq_m", "pq_ksub", "nnz")
    h = dict(zip(keys, fields))
    if h["version"] != VERSION:
        raise ValueError(f"version {h['version']}")
    if zlib.crc32(raw[:124]) != struct.unpack_from("<I", raw, 124)[0]:
        raise ValueError("header checksum")
    if any(raw[72:124]):
        raise ValueError("reserved header bytes")
    s = h["sections"]
    tab_end = HEADER + ENTRY * s
    if len(raw) < tab_end + 4:
        raise ValueError("truncated table")
    if zlib.crc32(raw[HEADER:tab_end]) != struct.unpack_from("<I", raw, tab_end)[0]:
        raise ValueError("table checksum")
    shapes = _shapes(h)
    out = {}
    end = tab_end + 4
    prev = 0
    for j in range(s):
        i, crc, off, size, zero = struct.unpack_from("<IIQQQ", raw, HEADER + ENTRY * j)
        # each section at the first 64-byte boundary after what precedes it
        if i not in SECTIONS or i <= prev or zero or off != _pad(end):
            raise ValueError(f"table entry {j}")
        if any(raw[end:min(off, len(raw))]):
            raise ValueError(f"padding before table entry {j}")
        name, dt = SECTIONS[i]
        shape = shapes[name]
        if size != int(np.prod(shape)) * np.dtype(dt).itemsize or size == 0:
            raise ValueError(f"{name} size")
        if off + size > len(raw):
            raise ValueError(f"{name} truncated")
        blob = raw[off:off + size]
        if zlib.crc32(blob) != crc:
            raise ValueError(f"{name} checksum")
        out[name] = np.frombuffer(blob, dtype=dt).reshape(shape)
        prev, end = i, off + size
    if end != len(raw):
        raise ValueError("trailing bytes")
    return h, out


def crc32(data):
    return zlib.crc32(data)
