"""Pins of the oracle's number formats against numpy / torch CPU casts."""
import numpy as np
import pytest
import torch

import oracle


def _samples(n=200_000, seed=0):
    rng = np.random.default_rng(seed)
    x = np.concatenate([
        rng.standard_normal(n).astype(np.float32),
        (rng.standard_normal(n) * 1e-5).astype(np.float32),        # subnormal fp16 range
        (rng.standard_normal(n) * 3e4).astype(np.float32),          # near fp16 overflow
        np.array([0.0, -0.0, 1.0, -1.0, 65504, 65519.99, 65520, -65520, 1e-8, 6e-8,
                  np.inf, -np.inf], np.float32),
    ])
    return x


def test_f16_matches_numpy():
    x = _samples()
    h = oracle.to_f16(x)
    ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(h, ref)
    back = oracle.from_f16(h)
    assert np.array_equal(back, ref.view(np.float16).astype(np.float32))


def test_bf16_matches_torch():
    x = _samples()
    b = oracle.to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(b, ref)
    # ties to even: 1 + 2^-8 rounds down, 1 + 3 * 2^-8 rounds up
    assert oracle.from_bf16(oracle.to_bf16(np.float32([1.00390625, 1.01171875]))).tolist() == \
        [1.0, 1.015625]


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 100_000), rng.standard_normal(100_000) * 0.01,
                        rng.standard_normal(100_000)]).astype(np.float32)
    e = oracle.to_e4m3(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(e, ref)
    back = oracle.from_e4m3(e)
    assert np.array_equal(back, torch.from_numpy(ref).view(torch.float8_e4m3fn).float().numpy())


def test_e4m3_saturates():
    # torch's cast is not saturating (480 -> NaN); the oracle clamps to +-448
    x = np.float32([448, 464, 480, 1e6, -1e6, np.inf, -np.inf])
    assert oracle.from_e4m3(oracle.to_e4m3(x)).tolist() == [448, 448, 448, 448, -448, 448, -448]


def test_e4m3_every_code_round_trips():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = oracle.from_e4m3(codes)
    back = oracle.to_e4m3(vals)
    zero = vals == 0
    assert np.array_equal(back[~zero], codes[~zero])
    # smallest subnormal, largest normal
    assert oracle.from_e4m3(np.uint8([1, 0x7E])).tolist() == [2.0 ** -9, 448.0]


def test_fp8_rows_scale():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((50, 64)).astype(np.float32) * 0.03
    X[3] = 0.0
    codes, scale = oracle.encode_fp8_rows(X)
    assert scale[3] == 1.0
    mx = np.abs(X).max(1)
    np.testing.assert_array_equal(scale[np.arange(50) != 3], (mx / np.float32(448))[np.arange(50) != 3])
    deq = oracle.from_e4m3(codes) * scale[:, None]
    # E4M3 keeps 3 mantissa bits: relative error <= 2^-4 for normal values
    big = np.abs(X) > scale[:, None] * 2.0 ** -6
    rel = np.abs(deq - X)[big] / np.abs(X)[big]
    assert rel.max() <= 2.0 ** -4 + 1e-7
    assert np.abs(oracle.from_e4m3(codes)).max() <= 448
