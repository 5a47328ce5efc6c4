"""Pins of the oracle's low-precision formats.

Decoders are checked over every bit pattern against library conversions
(numpy's binary16, torch's bfloat16 and float8_e4m3fn), and against values
typed in from the OCP FP8 specification; the E4M3 encoder is checked by
round trip over all finite codes, by ties-to-even at midpoints and against
torch's conversion on in-range random values.
"""
import os

import numpy as np
import torch

from oracle import lowp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_f16_decoder_all_patterns():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    got = lowp.f16_bits_to_f64(bits)
    ref = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def test_bf16_decoder_all_patterns():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    got = lowp.bf16_bits_to_f64(bits)
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def test_e4m3_decoder_all_patterns():
    bits = np.arange(256, dtype=np.uint16).astype(np.uint8)
    got = lowp.e4m3_bits_to_f64(bits)
    ref = torch.from_numpy(bits).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])
    assert nan.sum() == 2 and np.isnan(got[0x7F]) and np.isnan(got[0xFF])


def test_e4m3_spec_table():
    with open(os.path.join(GOLDEN, "e4m3_values.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for code, val in rows:
        c = int(code, 16)
        v = float(val)
        got = float(lowp.e4m3_bits_to_f64(np.array([c], dtype=np.uint8))[0])
        assert got == v and np.signbit(got) == np.signbit(v)
        enc = int(lowp.f64_to_e4m3_bits(np.array([v]))[0])
        assert enc == c


def test_e4m3_roundtrip_all_finite_codes():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    vals = lowp.e4m3_bits_to_f64(codes)
    assert np.array_equal(lowp.f64_to_e4m3_bits(vals), codes)


def test_e4m3_ties_to_even():
    # 1.0625 lies halfway between 1.0 (mantissa 000) and 1.125 (001): even is 1.0
    # 1.1875 lies halfway between 1.125 (001) and 1.25 (010): even is 1.25
    # 2**-10 lies halfway between 0 and the least subnormal 2**-9: even is 0
    # 3 * 2**-10 lies halfway between 2**-9 (001) and 2**-8 (010): even is 2**-8
    x = np.array([1.0625, 1.1875, 2.0 ** -10, 3 * 2.0 ** -10, -1.0625])
    got = lowp.e4m3_bits_to_f64(lowp.f64_to_e4m3_bits(x))
    assert np.array_equal(got, np.array([1.0, 1.25, 0.0, 2.0 ** -8, -1.0]))


def test_e4m3_encoder_matches_torch_in_range():
    g = np.random.default_rng(0)
    x = np.concatenate([g.uniform(-448, 448, 20000), g.standard_normal(20000) * 0.01,
                        g.standard_normal(20000)]).astype(np.float32)
    got = lowp.f64_to_e4m3_bits(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(got, ref)


def test_bf16_f16_rounding_matches_library():
    g = np.random.default_rng(1)
    x = (g.standard_normal(50000) * np.exp(g.uniform(-20, 20, 50000))).astype(np.float32)
    bf = lowp.f64_to_bf16_rne(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf, ref)
    y = x[np.abs(x) < 60000]
    h = lowp.f64_to_f16_rne(y.astype(np.float64))
    assert np.array_equal(h, y.astype(np.float16).astype(np.float64))


def test_quantize_properties():
    g = np.random.default_rng(2)
    x = g.standard_normal((64, 33)).astype(np.float32)
    q, s = lowp.quantize_e4m3(x)
    amax = np.max(np.abs(x))
    assert s == np.float32(amax / np.float32(448))
    deq = lowp.e4m3_bits_to_f64(q) * float(s)
    # the absmax element maps to +-448 (up to the rounding of x / s)
    i = np.unravel_index(np.argmax(np.abs(x)), x.shape)
    assert abs(lowp.e4m3_bits_to_f64(q)[i]) == 448.0
    # relative error of a normal e4m3 value is at most 2**-4; subnormal spacing is 2**-9
    err = np.abs(deq - x.astype(np.float64))
    assert np.all(err <= np.maximum(np.abs(x) * 2.0 ** -4, 2.0 ** -10 * float(s)) * 1.0001)
    # all-zero tensor: scale 1, codes 0
    qz, sz = lowp.quantize_e4m3(np.zeros((3, 3), np.float32))
    assert sz == 1.0 and np.all(qz == 0)


def test_quantize_non_finite_entries():
    """NaN and infinite entries become the NaN code with their sign (the
    format has no infinity); the finite entries keep the codes and the scale
    they would have without them."""
    g = np.random.default_rng(3)
    x = g.standard_normal((16, 9)).astype(np.float32)
    q0, s0 = lowp.quantize_e4m3(x)
    y = x.copy()
    y[1, 2], y[3, 4], y[5, 6], y[7, 8] = np.nan, np.inf, -np.inf, -np.nan
    q, s = lowp.quantize_e4m3(y)
    assert s == s0
    bad = ~np.isfinite(y)
    assert np.array_equal(q[~bad], q0[~bad])
    assert [int(v) for v in q[bad]] == [0x7F, 0x7F, 0xFF, 0xFF]
    assert np.all(np.isnan(lowp.e4m3_bits_to_f64(q[bad])))
    # a tensor with no finite nonzero entry keeps scale 1
    qn, sn = lowp.quantize_e4m3(np.array([[np.nan, 0.0], [np.inf, -0.0]], np.float32))
    assert sn == 1.0 and [int(v) for v in qn.ravel()] == [0x7F, 0x00, 0x7F, 0x80]
