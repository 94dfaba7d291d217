"""Index files on the host (no GPU): the library's reader and writer against
the oracle's independent writer and reader of the same documented format,
and every kind of damage the reader must reject with ANN_EFORMAT."""
import os
import struct
import zlib

import numpy as np
import pytest

import oracle
import oracle.index_file as oif
import synth

ann = pytest.importorskip("paper_2501_06121_amd")


@pytest.fixture(scope="module")
def dense():
    n, d = 600, 32
    X = synth.gaussian_mixture(5, n, d, 8, 0.3)
    g = oracle.hnsw_build(X, "l2", 8, 32, synth.level_uniforms(5, n))
    f8, s8 = oracle.encode_fp8_rows(X)
    sample, init = synth.pq_sample(5, n, n, 256)
    cb, _, _ = oracle.pq_train(X, 8, 256, sample, init, max_iter=2)
    codes = oracle.pq_encode(X, cb)
    arrays = dict(x_f32=X, x_f16=oracle.to_f16(X), x_bf16=oracle.to_bf16(X), x_fp8=f8,
                  fp8_scale=s8, pq_codebook=cb, pq_codes=codes)
    return dict(g=g, d=d, arrays=arrays)


@pytest.fixture(scope="module")
def sparse():
    n, vocab = 400, 300
    ip, ids, vals = synth.sparse_zipf(3, n, 12, vocab=vocab)
    g = oracle.hnsw_build_sparse(ip, ids, vals, vocab, 8, 32, synth.level_uniforms(3, n))
    return dict(g=g, d=vocab, arrays=dict(sp_indptr=ip, sp_ids=ids, sp_vals=vals))


def code_of(path):
    try:
        ann.ann_index_file_info(str(path))
    except ann.AnnError as e:
        return e.code, str(e)
    return ann.ANN_OK, ""


def test_crc32_is_the_documented_one():
    # the check value of CRC-32/IEEE (reflected 0xEDB88320, init and xor ~0)
    assert zlib.crc32(b"123456789") == 0xCBF43926


@pytest.mark.parametrize("which", ["dense", "sparse"])
def test_oracle_file_reads_in_the_library_and_both_writers_agree(tmp_path, dense, sparse, which):
    c = dense if which == "dense" else sparse
    metric = "l2" if which == "dense" else "ip"
    p_or, p_lib = tmp_path / "oracle.idx", tmp_path / "lib.idx"
    oif.write(p_or, c["g"], metric, c["d"], **c["arrays"])
    info = ann.ann_index_file_info(str(p_or))
    g = c["g"]
    assert (info["n"], info["d"], info["M"], info["M0"], info["max_level"], info["entry_point"]) == \
        (g.n, c["d"], g.M, g.M0, g.max_level, g.entry)
    assert info["metric"] == ann.METRIC[metric] and info["device"] == -1
    want_modes = {"dense": {"f32", "f16", "bf16", "fp8", "pq"}, "sparse": {"sparse"}}[which]
    assert info["modes"] == sum(1 << ann.MODE[m] for m in want_modes)
    # the library writes the same bytes for the same arrays
    ann.ann_index_save(str(p_lib), g, metric, c["d"], **c["arrays"])
    assert p_lib.read_bytes() == p_or.read_bytes()
    # and the oracle reads back every array
    h, arrs = oif.read(p_lib)
    assert h["n"] == g.n and h["sections"] == len(arrs)
    assert np.array_equal(arrs["levels"], g.levels) and np.array_equal(arrs["adj0"], g.adj0)
    assert np.array_equal(arrs["upper_off"], g.upper_off)
    for k, v in c["arrays"].items():
        assert np.array_equal(arrs[k], np.asarray(v).astype(arrs[k].dtype)), k


def sections_of(path):
    raw = path.read_bytes()
    s = struct.unpack_from("<I", raw, 12)[0]
    out = {}
    for j in range(s):
        i, crc, off, size, _ = struct.unpack_from("<IIQQQ", raw, 128 + 32 * j)
        out[oif.SECTIONS[i][0]] = (off, size)
    return out


def test_every_damaged_section_is_rejected(tmp_path, dense):
    p = tmp_path / "x.idx"
    oif.write(p, dense["g"], "l2", dense["d"], **dense["arrays"])
    good = p.read_bytes()
    assert code_of(p)[0] == ann.ANN_OK
    for name, (off, size) in sections_of(p).items():
        for pos in (off, off + size // 2, off + size - 1):
            bad = bytearray(good)
            bad[pos] ^= 0x10
            q = tmp_path / f"bad_{name}_{pos}.idx"
            q.write_bytes(bytes(bad))
            code, msg = code_of(q)
            assert code == ann.ANN_EFORMAT and name in msg and "checksum" in msg, (name, msg)


def test_header_and_table_damage(tmp_path, dense):
    p = tmp_path / "x.idx"
    oif.write(p, dense["g"], "l2", dense["d"], **dense["arrays"])
    good = p.read_bytes()

    def variant(tag, edit, fix_header_crc=False, fix_table_crc=False):
        b = bytearray(good)
        edit(b)
        if fix_header_crc:
            struct.pack_into("<I", b, 124, zlib.crc32(bytes(b[:124])))
        if fix_table_crc:
            s = struct.unpack_from("<I", b, 12)[0]
            struct.pack_into("<I", b, 128 + 32 * s, zlib.crc32(bytes(b[128:128 + 32 * s])))
        q = tmp_path / f"{tag}.idx"
        q.write_bytes(bytes(b))
        return code_of(q)

    def setb(pos, fmt, v):
        return lambda b: struct.pack_into(fmt, b, pos, v)

    cases = {
        "magic": (lambda b: b.__setitem__(slice(0, 8), b"ANNINDEY"), False, False, "magic"),
        "header crc": (setb(16, "<q", 601), False, False, "header checksum"),
        "version 2": (setb(8, "<I", 2), True, False, "version 2"),
        "version 0": (setb(8, "<I", 0), True, False, "version 0"),
        "reserved": (lambda b: b.__setitem__(100, 1), True, False, "reserved"),
        "section count": (setb(12, "<I", 15), True, False, "section count"),
        "n mismatch": (setb(16, "<q", 601), True, False, "bytes"),
        "d mismatch": (setb(24, "<i", 48), True, False, "bytes"),
        "table crc": (setb(128 + 16, "<Q", 1), False, False, "table checksum"),
        "unknown id": (setb(128, "<I", 99), False, True, "unknown section"),
        "misaligned": (lambda b: struct.pack_into("<Q", b, 128 + 8,
                                                  struct.unpack_from("<Q", b, 128 + 8)[0] + 8),
                       False, True, "misaligned"),
        "metric": (setb(28, "<i", 7), True, False, "metric"),
        "entry point": (setb(44, "<i", 10 ** 6), True, False, "entry point"),
    }
    for tag, (edit, fh, ft, words) in cases.items():
        code, msg = variant(tag.replace(" ", "_"), edit, fh, ft)
        assert code == ann.ANN_EFORMAT and words in msg, (tag, msg)


def test_truncated_and_padded_files(tmp_path, dense):
    p = tmp_path / "x.idx"
    oif.write(p, dense["g"], "l2", dense["d"], **dense["arrays"])
    good = p.read_bytes()
    secs = sections_of(p)
    cuts = {0, 1, 64, 127, 128, 200, len(good) - 1}
    for off, size in secs.values():
        cuts |= {off, off + size // 2}
    for cut in sorted(cuts):
        q = tmp_path / f"cut_{cut}.idx"
        q.write_bytes(good[:cut])
        code, msg = code_of(q)
        assert code == ann.ANN_EFORMAT, (cut, msg)
    q = tmp_path / "long.idx"
    q.write_bytes(good + b"\0" * 64)
    code, msg = code_of(q)
    assert code == ann.ANN_EFORMAT and "after the last section" in msg


def test_padding_and_section_placement(tmp_path, dense):
    """Sections start at the first 64-byte boundary after what precedes them,
    with zero bytes in between: a nonzero padding byte, or a section moved to
    a later boundary (table and checksums kept valid), is rejected by both
    readers."""
    p = tmp_path / "x.idx"
    oif.write(p, dense["g"], "l2", dense["d"], **dense["arrays"])
    good = p.read_bytes()
    s = struct.unpack_from("<I", good, 12)[0]
    table_end = 128 + 32 * s + 4
    gaps = [(table_end, min(off for off, _ in sections_of(p).values()))]
    ends = sorted((off + size, off) for off, size in sections_of(p).values())
    offs = sorted(off for off, _ in sections_of(p).values())
    gaps += [(e, nxt) for (e, _), nxt in zip(ends, offs[1:]) if nxt > e]
    assert any(b > a for a, b in gaps), "the fixture has no padding to damage"
    for a, b in gaps:
        if b <= a:
            continue
        bad = bytearray(good)
        bad[a] = 0x5A
        q = tmp_path / f"pad_{a}.idx"
        q.write_bytes(bytes(bad))
        code, msg = code_of(q)
        assert code == ann.ANN_EFORMAT and "padding" in msg, (a, msg)
        with pytest.raises(ValueError):
            oif.read(q)
    # the last section moved 64 bytes further, the gap zero-filled
    j = s - 1
    i, crc, off, size, _ = struct.unpack_from("<IIQQQ", good, 128 + 32 * j)
    bad = bytearray(good[:off]) + b"\0" * 64 + good[off:off + size]
    struct.pack_into("<Q", bad, 128 + 32 * j + 8, off + 64)
    struct.pack_into("<I", bad, 128 + 32 * s, zlib.crc32(bytes(bad[128:128 + 32 * s])))
    q = tmp_path / "moved.idx"
    q.write_bytes(bytes(bad))
    code, msg = code_of(q)
    assert code == ann.ANN_EFORMAT and "misplaced" in msg, msg
    with pytest.raises(ValueError):
        oif.read(q)


def test_inconsistent_contents_with_valid_checksums(tmp_path, dense, sparse):
    g = dense["g"]

    class G:
        pass

    def copy_graph(src):
        h = G()
        for k in ("n", "M", "M0", "max_level", "entry", "levels", "adj0", "upper_off", "upper_adj"):
            v = getattr(src, k)
            setattr(h, k, v.copy() if isinstance(v, np.ndarray) else v)
        return h

    bad = copy_graph(g)
    bad.adj0[3, 0] = g.n + 5                      # neighbour id out of range
    p = tmp_path / "ids.idx"
    oif.write(p, bad, "l2", dense["d"], **dense["arrays"])
    code, msg = code_of(p)
    assert code == ann.ANN_EFORMAT and "adj0" in msg
    bad = copy_graph(g)
    bad.levels = bad.levels.copy()
    bad.levels[bad.entry] = 0                      # entry point below max_level
    p = tmp_path / "entry.idx"
    oif.write(p, bad, "l2", dense["d"], **dense["arrays"])
    assert code_of(p)[0] == ann.ANN_EFORMAT
    # fp8 codes without their scales, and a sparse index under L2
    arr = dict(dense["arrays"])
    raw = oif.write
    p = tmp_path / "fp8.idx"
    raw(p, g, "l2", dense["d"], x_fp8=arr["x_fp8"], fp8_scale=arr["fp8_scale"])
    assert code_of(p)[0] == ann.ANN_OK
    b = bytearray(p.read_bytes())                  # drop the scale section from the table
    s = struct.unpack_from("<I", b, 12)[0]
    ids = [struct.unpack_from("<I", b, 128 + 32 * j)[0] for j in range(s)]
    assert ids[-1] == 9
    struct.pack_into("<I", b, 12, s - 1)
    struct.pack_into("<I", b, 124, zlib.crc32(bytes(b[:124])))
    struct.pack_into("<I", b, 128 + 32 * (s - 1), zlib.crc32(bytes(b[128:128 + 32 * (s - 1)])))
    off9 = struct.unpack_from("<Q", b, 128 + 32 * (s - 1) + 8)[0]
    q = tmp_path / "fp8_noscale.idx"
    q.write_bytes(bytes(b[:off9]))
    code, msg = code_of(q)
    assert code == ann.ANN_EFORMAT, msg
    p = tmp_path / "sparse_l2.idx"
    oif.write(p, sparse["g"], "l2", sparse["d"], **sparse["arrays"])
    code, msg = code_of(p)
    assert code == ann.ANN_EFORMAT and "inner product" in msg


def test_missing_file_and_null_arguments(tmp_path):
    code, msg = code_of(tmp_path / "nope.idx")
    assert code == ann.ANN_EINVAL and "cannot open" in msg
    L = ann.lib()
    assert L.ann_index_file_info(None, None) == ann.ANN_EINVAL
    assert L.ann_index_load(None, 0, None) == ann.ANN_EINVAL
    assert L.ann_index_save(None, None) == ann.ANN_EINVAL


def test_load_checks_the_file_before_the_device(tmp_path, dense):
    """Without a GPU a valid file gets as far as the device (ANN_ENODEV); a
    damaged one is rejected first (ANN_EFORMAT)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the no-GPU path")
    p = tmp_path / "x.idx"
    oif.write(p, dense["g"], "l2", dense["d"], **dense["arrays"])
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_load(str(p))
    assert e.value.code == ann.ANN_ENODEV
    b = bytearray(p.read_bytes())
    b[-1] ^= 1
    p.write_bytes(bytes(b))
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_load(str(p))
    assert e.value.code == ann.ANN_EFORMAT
