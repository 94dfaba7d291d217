"""GPU parity of the FP8-E4M3 row encoding against the oracle's, bit for bit
(codes and scales), including ties, the subnormal range, saturation, zero
rows and negative zero."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ann = pytest.importorskip("paper_2501_06121_amd")

pytestmark = pytest.mark.gpu


def check(X):
    codes, scale = ann.ann_encode_fp8(torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0"))
    torch.cuda.synchronize()
    rc, rs = oracle.encode_fp8_rows(X)
    assert np.array_equal(scale.cpu().numpy().view(np.uint32), rs.view(np.uint32))
    got = codes.cpu().numpy()
    assert np.array_equal(got, rc), np.argwhere(got != rc)[:5]


@pytest.mark.parametrize("d", [1, 7, 64, 96, 768, 1000])
def test_random_rows(d):
    rng = np.random.default_rng(d)
    X = (rng.standard_normal((300, d)) * np.exp(rng.uniform(-12, 12, (300, 1)))).astype(np.float32)
    check(X)


def test_vmf_rows():
    check(synth.dense_base(synth.WORKLOADS["vmf1m"], n=2000))


def test_edge_values():
    # rows whose quotients hit E4M3 ties, the subnormal range, the largest
    # value, zeros (whole rows too) and negative zero
    row_max = 448.0
    ties = [(8 + k + 0.5) * 2.0 ** e for e in range(-6, 8) for k in range(8)]
    sub = [k * 2.0 ** -10 for k in range(0, 20)]
    vals = np.array(ties + sub + [row_max, -row_max, 1e-30, -0.0, 0.0, 447.9, 300.0], np.float32)
    X = np.zeros((4, vals.size), np.float32)
    X[0] = vals
    X[1] = -vals
    X[2, 5] = -3.0          # one nonzero
    # row 3 all zero: scale 1, codes 0
    check(X)
