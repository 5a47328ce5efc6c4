"""Oracle (test infrastructure only): low-precision number formats, from their definitions.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The paper's evaluation uses FP16 inputs with FP32 accumulation (Performance
Evaluation section); the BF16 and FP8 inputs of this project extend that
precision ladder.  The paper fixes no rounding or scaling rule for them, so
the readings used here are:

* BF16 is the upper half of an IEEE binary32 word; a stored BF16 value is
  exactly the binary32 value whose low 16 bits are zero.
* FP16 is IEEE binary16 (1 sign, 5 exponent bits with bias 15, 10 fraction
  bits, subnormals, infinities and NaNs).
* FP8 is the OCP "E4M3FN" format (1 sign, 4 exponent bits with bias 7, 3
  fraction bits, subnormals, no infinities, NaN = exponent and fraction all
  ones, largest finite magnitude 448).
* Per-tensor FP8 quantisation: absmax = max |x| over the tensor,
  s = absmax / 448 rounded to binary32 (s = 1 when absmax is 0), and each code
  is q = RNE_e4m3(clamp(x / s, -448, 448)) with x / s rounded to binary32.
  The quantisation decision is taken in binary32, as on the device.

Every decoder maps a stored bit pattern to the exact float64 value it denotes;
every encoder works on exact float64 arithmetic (scaling by powers of two and
rounding half to even), so no library conversion routine is involved.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


# ---------------------------------------------------------------- decoders

def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Exact value of BF16 bit patterns (uint16) as float64."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def f16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Exact value of IEEE binary16 bit patterns (uint16) as float64, decoded field by field."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.int64)
    sign = np.where((b >> 15) & 1, -1.0, 1.0)
    exp = (b >> 10) & 0x1F
    frac = (b & 0x3FF).astype(np.float64)
    normal = sign * np.ldexp(1.0 + frac / 1024.0, (exp - 15).astype(np.int32))
    sub = sign * np.ldexp(frac / 1024.0, -14)
    special = np.where(frac == 0, sign * np.inf, np.nan)
    return np.where(exp == 0, sub, np.where(exp == 31, special, normal))


def e4m3_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Exact value of OCP E4M3FN bit patterns (uint8) as float64, decoded field by field."""
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    sign = np.where((b >> 7) & 1, -1.0, 1.0)
    exp = (b >> 3) & 0xF
    frac = (b & 0x7).astype(np.float64)
    normal = sign * np.ldexp(1.0 + frac / 8.0, (exp - 7).astype(np.int32))
    sub = sign * np.ldexp(frac / 8.0, -6)
    val = np.where(exp == 0, sub, normal)
    return np.where((exp == 15) & (frac == 7), np.nan, val)


# ---------------------------------------------------------------- encoders

def _rne_to_grid(a: np.ndarray, mant_bits: int, emin: int) -> np.ndarray:
    """Round non-negative float64 ``a`` to the nearest value of a binary format
    with ``mant_bits`` fraction bits and minimum normal exponent ``emin``
    (ties to even), ignoring overflow.  Returns the rounded float64 value."""
    a = np.asarray(a, dtype=np.float64)
    _, e2 = np.frexp(a)                      # a = f * 2**e2, f in [0.5, 1)
    e = np.maximum(e2.astype(np.int64) - 1, emin)   # floor(log2 a), clamped to subnormal range
    e = np.where(a == 0, emin, e)
    spacing_exp = (e - mant_bits).astype(np.int32)
    scaled = np.ldexp(a, -spacing_exp)       # exact: scaling by a power of two
    n = np.rint(scaled)                      # round half to even
    return np.ldexp(n, spacing_exp)


def f64_to_e4m3_bits(x: np.ndarray) -> np.ndarray:
    """Encode finite float64 values with |x| <= 448 to E4M3FN codes, rounding to
    nearest even.  Values outside the range must be clamped by the caller."""
    x = np.asarray(x, dtype=np.float64)
    if np.any(~np.isfinite(x)) or np.any(np.abs(x) > E4M3_MAX):
        raise ValueError("e4m3 encoder needs finite inputs clamped to [-448, 448]")
    neg = np.signbit(x)
    v = _rne_to_grid(np.abs(x), 3, -6)
    _, e2 = np.frexp(v)
    e = e2.astype(np.int64) - 1
    is_normal = v >= 2.0 ** -6
    exp_field = np.where(is_normal, e + 7, 0)
    mant_norm = np.ldexp(v, (-e).astype(np.int32)) - 1.0        # in [0, 1), multiple of 1/8
    mant_field = np.where(is_normal, np.rint(mant_norm * 8.0), np.rint(v * 2.0 ** 9))
    code = (exp_field.astype(np.int64) << 3) | mant_field.astype(np.int64)
    code = np.where(v == 0, 0, code)
    return (code | (neg.astype(np.int64) << 7)).astype(np.uint8)


def f64_to_bf16_rne(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value (ties to even) of float64 ``x`` in the normal/subnormal
    range of binary32, returned as float64 (overflow is not handled)."""
    x = np.asarray(x, dtype=np.float64)
    return np.copysign(_rne_to_grid(np.abs(x), 7, -126), x)


def f64_to_f16_rne(x: np.ndarray) -> np.ndarray:
    """Nearest binary16 value (ties to even) of float64 ``x``; overflow not handled."""
    x = np.asarray(x, dtype=np.float64)
    return np.copysign(_rne_to_grid(np.abs(x), 10, -14), x)


# ---------------------------------------------------------------- quantisation

def e4m3_scale(x_f32: np.ndarray) -> np.float32:
    """Per-tensor scale s = absmax / 448 in binary32 over the finite entries
    (1 when none of them is nonzero)."""
    x = np.asarray(x_f32, dtype=np.float32)
    fin = np.abs(x[np.isfinite(x)])
    amax = np.float32(np.max(fin)) if fin.size else np.float32(0)
    if amax == 0:
        return np.float32(1.0)
    return np.float32(amax) / np.float32(E4M3_MAX)


E4M3_NAN = 0x7F     # E4M3FN has no infinity; S.1111.111 is its NaN


def quantize_e4m3(x_f32: np.ndarray, scale: np.float32 | None = None):
    """Per-tensor FP8 quantisation.  Returns (codes uint8, scale float32).

    The quotient x / s is rounded to binary32 (numpy's float32 division is the
    correctly rounded IEEE operation), clamped to [-448, 448], then rounded to
    E4M3 with ties to even.  A NaN or infinite entry (which the format cannot
    hold; the paper's inputs are finite) becomes the NaN code with the
    entry's sign, and the scale is taken over the finite entries only, so
    such an entry shows up as NaN in the product instead of as a finite
    value."""
    x = np.asarray(x_f32, dtype=np.float32)
    s = e4m3_scale(x) if scale is None else np.float32(scale)
    fin = np.isfinite(x)
    with np.errstate(invalid="ignore", over="ignore"):
        y = (np.where(fin, x, np.float32(0)) / s).astype(np.float32)
    y = np.clip(y, np.float32(-E4M3_MAX), np.float32(E4M3_MAX))
    q = f64_to_e4m3_bits(y.astype(np.float64))
    nan_code = (E4M3_NAN | (np.signbit(x).astype(np.uint8) << 7)).astype(np.uint8)
    return np.where(fin, q, nan_code).astype(np.uint8), s


def decode(bits: np.ndarray, dtype: str) -> np.ndarray:
    """Exact float64 value of stored elements of the named type."""
    if dtype == "f32":
        return np.asarray(bits, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f64(bits)
    if dtype == "f16":
        return f16_bits_to_f64(bits)
    if dtype == "f8e4m3":
        return e4m3_bits_to_f64(bits)
    raise ValueError(dtype)
