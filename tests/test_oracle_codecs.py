"""Pins of the oracle's FP16 and FP8 (OCP E4M3FN) codecs and channel scale."""
import numpy as np
import pytest
import torch

import oracle


def test_f16_matches_numpy():
    rng = np.random.default_rng(31)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 5, 20000),
        np.array([0.0, -0.0, 65504.0, 65519.0, 65520.0, 70000.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26,
                  1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, -1.5, 2.0 ** -14]),
    ])
    # double -> binary16 in one rounding (numpy rounds directly from float64)
    with np.errstate(over="ignore"):                 # values past 65520 overflow to inf on purpose
        ref = x.astype(np.float16).view(np.uint16)
    got = oracle.f16_encode(x)
    assert np.array_equal(got, ref)
    codes = np.arange(65536, dtype=np.uint16)
    finite = ~np.isnan(codes.view(np.float16))
    np.testing.assert_array_equal(oracle.f16_decode(codes[finite]), codes[finite].view(np.float16).astype(np.float64))


def test_e4m3_hand_values():
    x = [448.0, 2.0 ** -9, 2.0 ** -6, 1.0, -1.0, 500.0, -1e6, 0.0, 1.0625, 1.1875, 2.0 ** -10, 3 * 2.0 ** -10, 464.0]
    want = [0x7E, 0x01, 0x08, 0x38, 0xB8, 0x7E, 0xFE, 0x00, 0x38, 0x3A, 0x00, 0x02, 0x7E]
    assert list(oracle.e4m3_encode(x)) == want
    assert oracle.e4m3_encode([float("nan")])[0] & 0x7F == 0x7F


def test_e4m3_matches_torch():
    rng = np.random.default_rng(32)
    x32 = np.concatenate([
        (rng.standard_normal(50000) * 2.0 ** rng.integers(-12, 9, 50000)).astype(np.float32),
        np.float32([0.0, 448.0, 440.0, 2.0 ** -9, 2.0 ** -10, 0.0029296875, 1.0625, 15.5, 240.0]),
    ])
    x32 = x32[np.abs(x32) <= 448.0]
    ref = torch.from_numpy(x32).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = oracle.e4m3_encode(x32.astype(np.float64))
    assert np.array_equal(got, ref)
    codes = np.arange(256, dtype=np.uint8)
    codes = codes[(codes & 0x7F) != 0x7F]
    dec = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.e4m3_decode(codes), dec)


def test_e4m3_scale():
    assert oracle.e4m3_scale(np.array([1.0, -3.0])) == 128.0      # 3 * 128 = 384 <= 448 < 768
    assert oracle.e4m3_scale(np.array([448.0])) == 1.0
    assert oracle.e4m3_scale(np.array([448.0001])) == 0.5
    assert oracle.e4m3_scale(np.zeros(4)) == 1.0
    assert oracle.e4m3_scale(np.array([0.875])) == 512.0           # 448 exactly
    rng = np.random.default_rng(33)
    for _ in range(200):
        x = rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3)
        s = oracle.e4m3_scale(x)
        m = np.abs(x).max()
        assert s * m <= 448.0 < 2 * s * m
        assert np.log2(s) == int(np.log2(s))
