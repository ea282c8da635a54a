"""Pins for the oracle's low-precision formats (oracle/quant.py).

The conversions are checked against an independent implementation, torch's
CPU casts to bfloat16 and float8_e4m3fn (both round to nearest even), on
random values and on the cases a plausible mistake would get wrong: exact
ties of both parities, subnormals, the top of the range, signed zero.
torch's float8 cast returns NaN from 464 up, where this format saturates to
448 by definition; that range is pinned to the definition instead.  The
decoders are checked on all 256 (FP8) byte patterns, the column-scaled form
by its error bound (half a unit in the last place of E4M3, relative 2^-4).
"""

import numpy as np
import pytest
import torch

from oracle import quant as Qz


def _samples(rng):
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-12, 4, 20000),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0, 2.0 ** -126, 2.0 ** -149, 3.4e38, -3.4e38]),
    ]).astype(np.float32)
    return x


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = _samples(rng)
    # exact ties: low 16 bits 0x8000 with even and odd kept bits
    ties = (rng.integers(0, 2 ** 31, 4000, dtype=np.uint64).astype(np.uint32) & 0xFFFF0000) | 0x8000
    x = np.concatenate([x, ties.view(np.float32)])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(Qz.bf16_bits(x), ref)
    assert np.array_equal(Qz.bf16_value(ref), torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy())


def test_e4m3_matches_torch_below_saturation():
    rng = np.random.default_rng(1)
    x = _samples(rng)
    x = x[np.abs(x) < 464.0]
    # ties between neighbouring E4M3 values of every binade, both parities
    grid = Qz.e4m3_value(np.arange(0, 0x7E, dtype=np.uint8)).astype(np.float64)
    mids = ((grid[:-1] + grid[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, -mids, np.float32([447.99, 448.0, 455.0, 463.9, 2.0 ** -10, 3 * 2.0 ** -10])])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(Qz.e4m3_bits(x), ref)


def test_e4m3_saturates_and_decodes():
    big = np.float32([448.0, 464.0, 1e6, np.inf])
    assert np.all(Qz.e4m3_bits(big) == 0x7E) and np.all(Qz.e4m3_bits(-big) == 0xFE)
    assert Qz.e4m3_bits(np.float32([np.nan]))[0] == 0x7F
    allb = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(allb).view(torch.float8_e4m3fn).float().numpy()
    val = Qz.e4m3_value(allb)
    assert np.array_equal(np.isnan(val), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(val[ok], ref[ok])
    assert np.array_equal(Qz.e4m3_bits(val[ok]), allb[ok])             # round trip, signed zero included


def test_fp8_column_scaling_error_bound():
    rng = np.random.default_rng(2)
    A = (rng.standard_normal((300, 50)) * np.logspace(-3, 2, 50)[None, :]).astype(np.float32)
    A[:, 7] = 0.0
    Aq, s = Qz.quantize_fp8(A)
    assert s[7] == 1.0 and np.all(Aq[:, 7] & 0x7F == 0)
    D = Qz.dequantize_fp8(Aq, s)
    scaled = np.abs(A.astype(np.float64)) / s[None, :]
    normal = scaled >= 2.0 ** -6
    err = np.abs(D - A.astype(np.float64))
    # half an ulp: 2^-4 relative for normals, 2^-10 * s absolute for subnormals (+ FP32 scaling rounding)
    assert np.all(err[normal] <= (2.0 ** -4 * 1.0001) * np.abs(A.astype(np.float64))[normal])
    assert np.all(err[~normal] <= 2.0 ** -10 * np.broadcast_to(s, A.shape)[~normal] * 1.0001)
    col_max = np.max(np.abs(Qz.e4m3_value(Aq)), axis=0)
    assert np.all(col_max[np.arange(50) != 7] == 448.0)


def test_bf16_dequantize_relative_error():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((100, 80)).astype(np.float32)
    D = Qz.dequantize_bf16(Qz.quantize_bf16(A))
    assert np.all(np.abs(D - A) <= 2.0 ** -8 * np.abs(A.astype(np.float64)))      # 8 significant bits
