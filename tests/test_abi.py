"""The C-ABI library: loads, exports every declared symbol, rejects bad
arguments on the host (no GPU needed for any of these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2501_06121_amd as ann

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ann.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(ann_\w+)\s*\(", text, flags=re.M))


def test_library_loads_and_exports_all_declared_symbols():
    L = ann.lib()
    decl = declared_functions()
    assert decl == set(ann.SIGNATURES), decl ^ set(ann.SIGNATURES)
    for name in decl:
        assert hasattr(L, name), name
    assert ann.ann_version() == 1


def test_struct_layouts_match_the_c_header(tmp_path):
    """ctypes mirrors vs. what gcc lays out from include/ann.h."""
    import subprocess
    structs = {"ann_index_desc": ann.AnnIndexDesc, "ann_batch": ann.AnnBatch,
               "ann_launch_cfg": ann.AnnLaunchCfg, "ann_info": ann.AnnIndexInfo,
               "ann_server_cfg": ann.AnnServerCfg, "ann_request": ann.AnnRequest,
               "ann_completion": ann.AnnCompletion, "ann_server_state": ann.AnnServerState, "ann_ivf_batch": ann.AnnIvfBatch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ann.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_null_arguments_rejected():
    L = ann.lib()
    out = C.c_void_p()
    assert L.ann_index_create(None, 0, C.byref(out)) == ann.ANN_EINVAL
    assert "NULL" in L.ann_last_error().decode()
    assert L.ann_search(None, None, 0, 10, 10, None, None) == ann.ANN_EINVAL
    assert L.ann_search_ex(None, None, None) == ann.ANN_EINVAL
    assert L.ann_index_free(None) == ann.ANN_OK
    assert L.ann_ivf_create(None, 4, None, None, None, C.byref(out)) == ann.ANN_EINVAL
    assert L.ann_ivf_search(None, None, None) == ann.ANN_EINVAL
    assert L.ann_ivf_free(None) == ann.ANN_OK


def test_pq_arguments_checked_on_the_host():
    """Shape and pointer checks of the device PQ entry points run before any
    device call (so they hold without a GPU)."""
    L = ann.lib()
    it = C.c_int32(0)
    # d not a multiple of m, subspaces wider than 32, ksub out of range, NULL pointers
    assert L.ann_pq_encode(None, 10, 100, None, 3, 256, None, None) == ann.ANN_EINVAL
    assert L.ann_pq_encode(None, 10, 128, None, 2, 256, None, None) == ann.ANN_EUNSUP
    assert L.ann_pq_encode(None, 10, 128, None, 16, 257, None, None) == ann.ANN_EINVAL
    assert L.ann_pq_encode(None, 10, 128, None, 16, 256, None, None) == ann.ANN_EINVAL
    assert "NULL" in L.ann_last_error().decode()
    assert L.ann_pq_train(None, 10, 128, None, 100, None, 16, 256, 5, None, C.byref(it), None) == ann.ANN_EINVAL
    x = np.zeros(4, np.float32)
    p = x.ctypes.data
    assert L.ann_pq_train(p, 10, 128, p, 100, p, 16, 256, 5, p, C.byref(it), None) == ann.ANN_EINVAL
    assert "sample" in L.ann_last_error().decode()          # 100 sample points for 256 centroids
    assert L.ann_pq_train(p, 10, 128, p, 300, p, 16, 256, 0, p, C.byref(it), None) == ann.ANN_EINVAL


class _G:
    def __init__(self, n, M=4, M0=8):
        self.n, self.M, self.M0, self.max_level, self.entry = n, M, M0, 0, 0
        self.levels = np.zeros(n, np.uint8)
        self.adj0 = np.full((n, M0), -1, np.int32)
        for v in range(n):
            self.adj0[v, 0] = (v + 1) % n
        self.upper_off = np.full(n, -1, np.int32)
        self.upper_adj = np.zeros((0, M), np.int32)


def test_malformed_graphs_rejected_before_device_use():
    X = np.zeros((8, 16), np.float32)
    g = _G(8)
    g.adj0[3, 0] = 99                     # id out of range
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_create(g, "l2", 16, x_f32=X)
    assert e.value.code == ann.ANN_EFORMAT
    g = _G(8)
    g.adj0[2, :2] = [-1, 4]               # valid id after padding
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_create(g, "l2", 16, x_f32=X)
    assert e.value.code == ann.ANN_EFORMAT
    g = _G(8)
    g.levels[5] = 1                       # above max_level
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_create(g, "l2", 16, x_f32=X)
    assert e.value.code == ann.ANN_EFORMAT
    with pytest.raises(ann.AnnError) as e:  # d not a multiple of 16
        ann.ann_index_create(_G(8), "l2", 12, x_f32=np.zeros((8, 12), np.float32))
    assert e.value.code == ann.ANN_EFORMAT


@pytest.mark.skipif(ann.ann_device_count() > 0, reason="checks the no-GPU path")
def test_no_device_reported():
    with pytest.raises(ann.AnnError) as e:
        ann.ann_index_create(_G(8), "l2", 16, x_f32=np.zeros((8, 16), np.float32))
    assert e.value.code == ann.ANN_ENODEV


def test_server_rejects_bad_arguments_on_the_host():
    L = ann.lib()
    out = C.c_void_p()
    cfg = ann.AnnServerCfg(0, 0, 16, 16, 2, 10, 64, 100, 1 << 30)
    assert L.ann_server_create(None, C.byref(cfg), C.byref(out)) == ann.ANN_EINVAL
    assert L.ann_server_submit(None, None) == ann.ANN_EINVAL
    assert L.ann_server_poll(None, None, 0) == -ann.ANN_EINVAL
    assert L.ann_server_destroy(None) == ann.ANN_OK


def test_ivf_group_matches_the_oracle_grouping():
    """ann_ivf_group is host code: the lists of an assignment, ids ascending."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(9)
    for n, nlist in ((0, 3), (1, 1), (1000, 7), (5000, 300)):
        a = rng.integers(0, nlist, n).astype(np.int32)
        off, ids = ann.ann_ivf_group(a, nlist)
        roff, rids = oracle.ivf_lists(a, nlist)
        assert np.array_equal(off, roff) and np.array_equal(ids, rids)
    with pytest.raises(ann.AnnError) as e:
        ann.ann_ivf_group(np.array([0, 2], np.int32), 2)
    assert e.value.code == ann.ANN_EINVAL
