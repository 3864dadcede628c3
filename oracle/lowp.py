"""Oracle of the reduced-precision descriptor forms (BF16, FP8 E4M3 with a
per-descriptor scale) and of what the quantised matchers guarantee.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper matches real-valued descriptors by Euclidean distance (Sec. 2.4,
Eq. 6); the quantised forms are a precision variant of that contraction. Both
roundings are written here from the format definitions, in double precision:

  BF16      1 sign, 8 exponent, 7 stored mantissa bits (FP32's exponent range):
            a finite x = f 2^e with f in [0.5, 1) rounds to rint(f 2^8) 2^(e-8),
            ties to even (np.rint); below 2^-126 the grid is 2^-133.
  FP8 E4M3  (OCP "fn" form) 1 sign, 4 exponent bits (bias 7), 3 mantissa bits,
            no infinities: normals f 2^e with 2^-6 <= |x| <= 448 round to
            rint(f 2^4) 2^(e-4); below 2^-6 the grid is 2^-9 (subnormals);
            ties to even; values are saturated to +-448 before rounding.

Per-descriptor scale of the FP8 form (reading): m = max_k |d_k| and
s = m / 448 are FP32 values; each element is formed as v fl32(448 / m), i.e.
the FP32 product with the rounded reciprocal scale (not v / s), clamped to
[-448, 448] in FP32 and then rounded to E4M3; a zero row keeps s = 1. The
FP32 steps that decide a code are taken in FP32 (numpy float32), as the kernel
takes them; only the final rounding is the format's.

Pins (tests/test_oracle_lowp.py): hand-built values (exactly representable
inputs, halves to even, the subnormal boundary, saturation), torch's own CPU
bfloat16 / float8_e4m3fn conversions on random inputs, byte decoding of known
E4M3 and BF16 codes, power-of-two gain invariance of the scaled form, and a
brute-force check of the recall guarantee on tiny sets.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

FP8_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """Nearest BF16 value of each FP32 input (round half to even), as float64."""
    v = np.asarray(x, dtype=np.float32).astype(np.float64)
    out = np.empty_like(v)
    tiny = np.abs(v) < 2.0 ** -126
    f, e = np.frexp(v[~tiny])
    out[~tiny] = np.ldexp(np.rint(np.ldexp(f, 8)), e - 8)
    out[tiny] = np.ldexp(np.rint(np.ldexp(v[tiny], 133)), -133)
    return out


def e4m3_round(x) -> np.ndarray:
    """Nearest E4M3 value of each input (round half to even, saturated at
    +-448), as float64."""
    v = np.clip(np.asarray(x, dtype=np.float64), -FP8_MAX, FP8_MAX)
    out = np.empty_like(v)
    sub = np.abs(v) < 2.0 ** -6
    out[sub] = np.ldexp(np.rint(np.ldexp(v[sub], 9)), -9)
    f, e = np.frexp(v[~sub])
    out[~sub] = np.ldexp(np.rint(np.ldexp(f, 4)), e - 4)
    return np.clip(out, -FP8_MAX, FP8_MAX)


def decode_e4m3(codes) -> np.ndarray:
    """Values of E4M3 bytes (sign, 4-bit exponent with bias 7, 3-bit mantissa;
    exponent 0 is subnormal m 2^-9; S.1111.111 is NaN)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    ex = (c >> 3) & 0xF
    man = c & 0x7
    val = np.where(ex == 0, man * 2.0 ** -9, (1.0 + man / 8.0) * np.ldexp(1.0, ex - 7))
    val = np.where((ex == 0xF) & (man == 0x7), np.nan, val)
    return sign * val


def decode_bf16(bits) -> np.ndarray:
    """Values of BF16 bit patterns (the upper half of an FP32 word)."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def quantize_bf16(desc_f32) -> np.ndarray:
    """BF16 form of FP32 descriptors [n, 128] (values, float64)."""
    return bf16_round(desc_f32)


def quantize_fp8(desc_f32) -> Tuple[np.ndarray, np.ndarray]:
    """FP8 E4M3 form of FP32 descriptors [n, 128] with one scale per row:
    (values q, float64 [n, 128]; scales s, float32 [n]); the descriptor is
    represented by s * q."""
    d = np.asarray(desc_f32, dtype=np.float32)
    m = np.abs(d).max(axis=1) if d.shape[0] else np.zeros(0, np.float32)
    pos = m > 0
    with np.errstate(divide="ignore"):
        s = np.where(pos, m / np.float32(FP8_MAX), np.float32(1.0)).astype(np.float32)
        inv = np.where(pos, np.float32(FP8_MAX) / np.where(pos, m, np.float32(1.0)),
                       np.float32(1.0)).astype(np.float32)
    x = np.clip(d * inv[:, None], np.float32(-FP8_MAX), np.float32(FP8_MAX)).astype(np.float32)
    return e4m3_round(x), s


def quantized_rows(desc_f32, precision: int) -> np.ndarray:
    """The descriptors as the quantised contraction sees them (float64):
    BF16 values (precision 1) or s * E4M3 values (precision 2)."""
    if precision == 1:
        return quantize_bf16(desc_f32)
    if precision == 2:
        q, s = quantize_fp8(desc_f32)
        return q * s.astype(np.float64)[:, None]
    raise ValueError("precision must be 1 (BF16) or 2 (FP8 E4M3)")


def quantized_scores(A32, B32, precision: int) -> np.ndarray:
    """Ranking score of every (query, candidate) pair under the quantised
    contraction, in double: |b|^2 - 2 a~.b~ with |b|^2 from the FP32
    descriptor and a~, b~ the quantised rows. Within a query, a smaller score
    is a nearer candidate; |a|^2 is constant per query and left out."""
    A = np.asarray(A32, np.float32)
    B = np.asarray(B32, np.float32)
    qa = quantized_rows(A, precision)
    qb = quantized_rows(B, precision)
    nb = (B.astype(np.float64) ** 2).sum(axis=1)
    return nb[None, :] - 2.0 * (qa @ qb.T)


def recall_guaranteed(scores: np.ndarray, j1: np.ndarray, j2: np.ndarray,
                      delta: float) -> Dict[str, np.ndarray]:
    """Queries whose true nearest candidates a quantised matcher must find
    when it rescores (at least) the two best candidates by its ranking score
    and knows that score within +-delta/2 of the values here.
    "j1": the true nearest j1 ranks first or second with a margin: fewer than
    two other candidates come within delta of it. "j1_j2": j1 and the true
    second nearest j2 both lead every other candidate by more than delta.
    scores: [nA, nB] from quantized_scores; j1, j2: the exact nearest and
    second-nearest candidates (-1 when absent)."""
    nA, nB = scores.shape
    g1 = np.zeros(nA, bool)
    g12 = np.zeros(nA, bool)
    for i in range(nA):
        a, b = int(j1[i]), int(j2[i])
        if a < 0:
            continue
        row = scores[i]
        others = np.sort(np.delete(row, a))
        g1[i] = others.size < 2 or row[a] + delta < others[1]
        if b < 0:
            g12[i] = g1[i]
            continue
        rest = np.delete(row, [a, b])
        g12[i] = rest.size == 0 or max(row[a], row[b]) + delta < rest.min()
    return {"j1": g1, "j1_j2": g12}
