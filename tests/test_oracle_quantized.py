"""Pins of the uint8 descriptor oracle (oracle/quantized.py)."""
import math

import numpy as np
from scipy.spatial.distance import cdist

from oracle import quantized as Q


def test_quantize_closed_forms():
    d = np.array([0.0, 1 / 1024, 3 / 1024, 5 / 1024, 0.1, 0.2, 0.4980468, 0.5, 1.0, -0.0],
                 np.float32)
    q = Q.quantize_u8(d)
    # 0.5 -> 0 and 2.5 -> 2 (halves to even), 1.5 -> 2, 51.2 -> 51, 102.4 -> 102,
    # 254.99 -> 255, 256 and 512 clamp to 255
    assert q.tolist() == [0, 0, 2, 2, 51, 102, 255, 255, 255, 0]
    assert q.dtype == np.uint8


def test_match_u8_against_cdist():
    rng = np.random.default_rng(3)
    A = rng.integers(0, 256, (40, 128)).astype(np.uint8)
    B = rng.integers(0, 256, (55, 128)).astype(np.uint8)
    B[9] = B[30]                                         # an exact duplicate row
    A[0] = B[30]
    o = Q.match_u8(A, B, ratio=0.8)
    D = cdist(A.astype(np.float64), B.astype(np.float64), "sqeuclidean")
    assert np.array_equal(o["j1"], D.argmin(axis=1))
    Ds = np.sort(D, axis=1)
    assert np.array_equal(o["D1"], Ds[:, 0].astype(np.int64))
    assert np.array_equal(o["D2"], Ds[:, 1].astype(np.int64))
    assert o["j1"][0] == 9 and o["D1"][0] == 0 and o["D2"][0] == 0 and o["match"][0] == -1
    keep = np.sqrt(Ds[:, 0]) < 0.8 * np.sqrt(Ds[:, 1])
    keep[0] = False
    assert np.array_equal(o["match"] >= 0, keep)
    assert np.allclose(o["d1"], np.sqrt(Ds[:, 0]) / 512, rtol=1e-15)


def test_match_u8_ratio_boundary_and_degenerate():
    A = np.zeros((1, 128), np.uint8)
    B = np.zeros((2, 128), np.uint8)
    B[0, 0] = 4                                          # D1 = 16 -> 4
    B[1, 1] = 5                                          # D2 = 25 -> 5: 4 < 0.8*5 is false
    assert Q.match_u8(A, B)["match"][0] == -1
    assert Q.match_u8(A, B, ratio=math.inf)["match"][0] == 0
    assert Q.match_u8(A, B, ratio=math.inf, abs_thresh=4 / 512)["match"][0] == -1
    o = Q.match_u8(A, B[:1])
    assert o["match"][0] == 0 and np.isinf(o["d2"][0])
    o = Q.match_u8(A, B[:0])
    assert o["match"][0] == -1 and o["j1"][0] == -1
