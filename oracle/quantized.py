"""FP64/integer oracle of the uint8 descriptor variant.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Descriptors of Sec. 2.3 are quantised the way SIFT implementations store them:
q = min(255, round(512 d)) per element (round half to even), from the FP32
descriptor values (the decision is taken on the same FP32 numbers on both
sides). Matching uint8 descriptors follows Eq. 6 with exact integer squared
distances D = sum (qa - qb)^2: the nearest registered row (lowest index on
ties) and the second smallest D over the others; distances are reported as
sqrt(D) / 512 (the scale of the float descriptors) and the query is kept when
sqrt(D1) < ratio sqrt(D2) in FP64 (ratio = +inf: no ratio test) and
sqrt(D1) / 512 < abs_thresh.
Pins (tests/test_oracle_quantized.py): closed-form quantisation values
(halves to even, clamping), integer distances against SciPy cdist on small
sets, the exact (4, 5) ratio case and index ties.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np


def quantize_u8(desc_f32: np.ndarray) -> np.ndarray:
    d = np.asarray(desc_f32, dtype=np.float32).astype(np.float64)
    return np.minimum(255.0, np.rint(512.0 * d)).astype(np.uint8)


def match_u8(qa: np.ndarray, qb: np.ndarray, ratio: float = 0.8,
             abs_thresh: float = math.inf) -> Dict[str, np.ndarray]:
    A = np.asarray(qa, np.int64)
    B = np.asarray(qb, np.int64)
    nA, nB = len(A), len(B)
    out = {"j1": np.full(nA, -1, np.int32), "D1": np.zeros(nA, np.int64),
           "D2": np.full(nA, -1, np.int64), "d1": np.full(nA, np.inf), "d2": np.full(nA, np.inf),
           "match": np.full(nA, -1, np.int32)}
    for i in range(nA):
        if nB == 0:
            continue
        D = ((B - A[i]) ** 2).sum(axis=1)
        j1 = int(np.argmin(D))                      # lowest index among equal minima
        out["j1"][i] = j1
        out["D1"][i] = D[j1]
        out["d1"][i] = math.sqrt(D[j1]) / 512.0
        if nB >= 2:
            rest = np.delete(D, j1)
            out["D2"][i] = rest.min()
            out["d2"][i] = math.sqrt(out["D2"][i]) / 512.0
        s1 = math.sqrt(float(D[j1]))
        s2 = math.sqrt(float(out["D2"][i])) if nB >= 2 else math.inf
        ratio_ok = math.isinf(ratio) or s1 < ratio * s2
        if ratio_ok and s1 / 512.0 < abs_thresh:
            out["match"][i] = j1
    return out
