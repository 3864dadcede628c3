"""Pins of the reduced-precision oracle (oracle/lowp.py): the BF16 and FP8 E4M3
roundings against hand-built values from the format definitions and against
torch's own CPU conversions, byte decoding of known codes, the per-descriptor
FP8 scale, and the recall guarantee against brute force on tiny sets."""
import math

import numpy as np
import pytest

from oracle import lowp


def f32(v):
    return np.float32(v)


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (-2.5, -2.5), (1.0 + 2 ** -7, 1.0 + 2 ** -7),          # representable
    (1.0 + 2 ** -8, 1.0),                                               # half: to even (down)
    (1.0 + 3 * 2 ** -8, 1.0 + 2 ** -6),                                  # half: to even (up)
    (1.0 + 2 ** -8 + 2 ** -20, 1.0 + 2 ** -7),                           # above half
    (-(1.0 + 3 * 2 ** -8), -(1.0 + 2 ** -6)),
    (3.0 * 2 ** -130, 3.0 * 2 ** -130),                                  # subnormal, exact
    (2 ** -133 + 2 ** -134, 2 ** -132),                                  # subnormal half: to even
    (2 ** -134, 0.0),                                                    # half of the smallest
    (0.1, 0.10009765625),
])
def test_bf16_hand_values(x, want):
    got = lowp.bf16_round(np.array([x], np.float32))[0]
    assert got == want


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (448.0, 448.0), (-448.0, -448.0), (240.0, 240.0),       # representable
    (1.0625, 1.0),            # half between 1 (mantissa 000) and 1.125 (001): even
    (1.1875, 1.25),           # half between 1.125 (001) and 1.25 (010): even
    (232.0, 224.0),           # half between 224 (110) and 240 (111): even
    (500.0, 448.0), (-1e6, -448.0),                                      # saturation
    (2 ** -9, 2 ** -9),       # smallest subnormal
    (2 ** -10, 0.0),          # half of it: ties to even (zero)
    (3 * 2 ** -10, 2 ** -8),  # half between 1 and 2 subnormal steps: even (2)
    (15 * 2 ** -10, 2 ** -6), # half between 7 steps (odd) and the smallest normal
    (2 ** -6, 2 ** -6),       # smallest normal
    (0.3, 0.3125),
])
def test_e4m3_hand_values(x, want):
    assert lowp.e4m3_round(np.array([x]))[0] == want


def test_decode_known_codes():
    assert lowp.decode_e4m3([0x7E, 0x38, 0x01, 0x08, 0x00, 0xB8, 0x77])[:7].tolist() == \
        [448.0, 1.0, 2 ** -9, 2 ** -6, 0.0, -1.0, 240.0]
    assert math.isnan(lowp.decode_e4m3([0x7F])[0]) and math.isnan(lowp.decode_e4m3([0xFF])[0])
    assert lowp.decode_bf16([0x3F80, 0xC020, 0x0001, 0x7F7F]).tolist() == \
        [1.0, -2.5, 2.0 ** -133, float(np.float32(3.3895313892515355e38))]


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(300_000) * np.exp(rng.uniform(-95, 85, 300_000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(lowp.bf16_round(x), want)


def test_e4m3_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = (rng.uniform(-448, 448, 300_000) * np.exp(rng.uniform(-16, 0, 300_000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(lowp.e4m3_round(x), want)
    # every code's value is its own rounding (the grid is closed)
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    v = lowp.decode_e4m3(codes)
    assert np.array_equal(lowp.e4m3_round(v), v)


def test_fp8_scale_and_codes():
    d = np.zeros((4, 128), np.float32)
    d[0, 0], d[0, 1], d[0, 2] = 0.2, 0.1, 0.05          # max 0.2
    d[1, :] = 0.0                                        # zero row: s = 1, codes 0
    d[2, 0], d[2, 5] = 448.0, 1.0625                    # s = 1, inv = 1: plain rounding
    d[3, 0], d[3, 1] = -3.0, 1.5
    q, s = lowp.quantize_fp8(d)
    assert s.dtype == np.float32
    assert s[0] == np.float32(np.float32(0.2) / np.float32(448.0))
    assert s[1] == 1.0 and np.all(q[1] == 0)
    assert s[2] == 1.0 and q[2, 0] == 448.0 and q[2, 5] == 1.0
    # the row maximum maps to (at most a rounding away from) 448
    assert q[0, 0] == 448.0 and q[3, 0] == -448.0
    # 1.5 / 3 * 448 = 224 exactly
    assert q[3, 1] == 224.0
    # x = v fl(448 / m) in FP32, then E4M3
    inv = np.float32(448.0) / np.float32(0.2)
    assert q[0, 1] == lowp.e4m3_round(np.float32(np.float32(0.1) * inv))


def test_fp8_power_of_two_gain_invariance():
    rng = np.random.default_rng(3)
    d = np.abs(rng.standard_normal((50, 128))).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q, s = lowp.quantize_fp8(d)
    for k in (-3, 1, 5):
        q2, s2 = lowp.quantize_fp8((d * np.float32(2.0 ** k)).astype(np.float32))
        assert np.array_equal(q, q2)
        assert np.array_equal(s2, (s * np.float32(2.0 ** k)).astype(np.float32))


def test_quantized_rows_error_bounds():
    rng = np.random.default_rng(4)
    d = np.abs(rng.standard_normal((200, 128))).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    b = lowp.quantized_rows(d, 1)
    assert np.all(np.abs(b - d) <= 2.0 ** -8 * np.abs(d))            # unit roundoff, 8 bits
    f = lowp.quantized_rows(d, 2)
    s = np.abs(d).max(axis=1, keepdims=True) / 448.0
    # normals: unit roundoff of 4 bits; subnormals: half of 2^-9 in scaled
    # units (plus the FP32 scaling product's own rounding)
    assert np.all(np.abs(f - d) <= np.maximum(2.0 ** -4 * np.abs(d), 2.0 ** -10 * s) * 1.0001)
    assert np.abs(f - d).max() > 2.0 ** -6 * np.abs(d).max() / 8   # FP8 is really coarser


def test_recall_guarantee_brute_force():
    """On tiny sets, every candidate perturbation within +-delta/2 keeps the
    guaranteed candidates within the two best by the perturbed score."""
    rng = np.random.default_rng(5)
    for trial in range(200):
        nA, nB = 3, int(rng.integers(1, 6))
        S = rng.integers(0, 6, (nA, nB)).astype(np.float64) * 0.25
        j1 = np.argmin(S, axis=1)
        j2 = np.array([np.argsort(S[i], kind="stable")[1] if nB > 1 else -1 for i in range(nA)])
        delta = 0.3
        g = lowp.recall_guaranteed(S, j1, j2, delta)
        for _ in range(20):
            P = S + rng.uniform(-delta / 2, delta / 2, S.shape)
            top2 = [set(np.argsort(P[i], kind="stable")[:2].tolist()) for i in range(nA)]
            for i in range(nA):
                if g["j1"][i]:
                    assert j1[i] in top2[i]
                if g["j1_j2"][i] and j2[i] >= 0:
                    assert {j1[i], j2[i]} == top2[i]
