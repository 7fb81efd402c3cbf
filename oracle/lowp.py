"""Reduced-precision operand rounding for the precision form of the passes
(test infrastructure only; see the package docstring).

The paper runs every product in float64 (Sec. 6).  The precision form runs the
v - 1 passes of Alg. 7 on rounded copies of both operands, accumulates exactly
(float64 here), and keeps the final product with A (Alg. 5 step 3, Alg. 9
step 2) exact.  The rounding rules are the published number formats:

  * bfloat16: the upper 16 bits of an IEEE binary32 value, round to nearest,
    ties to even, on the discarded 16 bits.
  * FP8 E4M3 ("e4m3fn" of the OCP 8-bit floating point specification): sign,
    4 exponent bits with bias 7, 3 mantissa bits; subnormal spacing 2^-9,
    largest finite value 448, no infinities; round to nearest, ties to even.
  * Block scaling (per tile of 32 consecutive entries along the contraction
    axis, the shared-scale block of the OCP microscaling formats): each block
    is divided by a power of two 2^e, e the smallest integer with
    max|x| / 2^e <= 448, before E4M3 rounding; 2^e is an E8M0 scale.  An
    all-zero block takes e = -127.

Pins (tests/test_oracle_pins.py): bfloat16 and E4M3 rounding bit-for-bit
against PyTorch's CPU conversions on random and special values; the minimality
of the block exponent; the half-spacing error bound; the invariance of the
precision-form basis under sub-half-ulp perturbations of A and Omega; and the
record of which operands the precision form rounds.
"""

from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0
MX_BLOCK = 32


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of bfloat16(x) for float32 x (round to nearest
    even; NaN stays NaN with the quiet bit set)."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return r.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """float64 values of bfloat16 bit patterns."""
    u = (np.asarray(bits, dtype=np.uint32) << 16).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray, axis: int | None = None) -> np.ndarray:
    """bfloat16 rounding of the float32 value of x, as float64 (axis unused:
    the format has no blocks)."""
    return bf16_value(bf16_bits(np.asarray(x, dtype=np.float32)))


def e4m3_round(y: np.ndarray) -> np.ndarray:
    """Round float64 values with |y| <= 448 to the nearest E4M3 value (ties
    to even), returned as float64."""
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    if np.any(a > E4M3_MAX):
        raise ValueError("e4m3_round expects |y| <= 448 (scale first)")
    # spacing of the grid at a: 2^-9 below 2^-6 (subnormals), else 2^(E-3)
    E = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    E = np.maximum(E, -6.0)
    spacing = np.exp2(E - 3.0)
    q = np.round(a / spacing) * spacing          # numpy rounds halves to even
    return np.copysign(q, y)


def e4m3_bits(q: np.ndarray) -> np.ndarray:
    """uint8 codes of values already on the E4M3 grid."""
    q = np.asarray(q, dtype=np.float64)
    s = (np.signbit(q)).astype(np.uint8) << 7
    a = np.abs(q)
    out = np.zeros(a.shape, dtype=np.uint8)
    sub = a < 2.0 ** -6
    out[sub] = np.round(a[sub] / 2.0 ** -9).astype(np.uint8)
    nz = ~sub
    E = np.floor(np.log2(a[nz])).astype(np.int64)
    mant = np.round(a[nz] / np.exp2(E) * 8.0).astype(np.int64) - 8
    out[nz] = ((E + 7) << 3 | mant).astype(np.uint8)
    return out | s


def mx_exponents(x: np.ndarray, axis: int) -> np.ndarray:
    """Block exponents e (int) for blocks of 32 consecutive entries of x along
    `axis` (the last block may be short): the smallest e with
    max|x| / 2^e <= 448, but at least -127; -127 for an all-zero block."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    K = x.shape[-1]
    nb = (K + MX_BLOCK - 1) // MX_BLOCK
    pad = nb * MX_BLOCK - K
    xp = np.concatenate([np.abs(x), np.zeros(x.shape[:-1] + (pad,))], axis=-1)
    amax = xp.reshape(x.shape[:-1] + (nb, MX_BLOCK)).max(axis=-1)
    e = np.full(amax.shape, -127, dtype=np.int64)
    nz = amax > 0
    # frexp gives amax/448 = f 2^t with f in [0.5, 1): e = t, or t - 1 when f == 0.5
    f, t = np.frexp(amax[nz] / E4M3_MAX)
    e[nz] = np.where(f == 0.5, t - 1, t)
    return np.maximum(e, -127)        # E8M0 holds 2^-127 .. 2^127


def round_mx_e4m3(x: np.ndarray, axis: int) -> np.ndarray:
    """Block-scaled E4M3 rounding of the float32 value of x, blocks of 32
    along `axis` (the contraction axis of the product it feeds), returned as
    float64 dequantized values q * 2^e."""
    x32 = np.asarray(x, dtype=np.float32).astype(np.float64)
    e = mx_exponents(x32, axis)
    xm = np.moveaxis(x32, axis, -1)
    scale = np.exp2(np.repeat(e, MX_BLOCK, axis=-1)[..., :xm.shape[-1]].astype(np.float64))
    q = e4m3_round(xm / scale) * scale
    return np.moveaxis(q, -1, axis)


ROUNDINGS = {
    "fp32": None,
    "bf16": round_bf16,
    "fp8_e4m3": round_mx_e4m3,
}
