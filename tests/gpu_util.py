"""Helpers shared by the GPU parity tests: device transfer, comparison rules."""
import math
import sys

import numpy as np

import oracle


def say(*a):
    """Name the case on stderr before a GPU step, flushed, so a crash log shows it."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_dev(img, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(img)).to(device)


def kp_numpy(kp):
    return {k: v.cpu().numpy() for k, v in kp.items()}


def assert_keypoints_equal(g, o):
    """Bit-exact integer fields; contrast is a correctly rounded FP32 quotient
    of exact integers, so it equals the FP64 value to FP32 rounding."""
    for f in ("x", "y", "scale", "type", "value"):
        assert np.array_equal(g[f].astype(np.int64), o[f].astype(np.int64)), f
    assert np.allclose(g["contrast"], o["contrast"], rtol=2e-7, atol=1e-9)


def orientation_ambiguity(hist):
    """Relative gap between the highest smoothed bin and the highest bin not
    adjacent to it. Adjacent near-ties move theta0 continuously (the two
    parabolas meet), so only non-adjacent near-ties can flip it."""
    k = np.argmax(hist, axis=1)
    h1 = hist[np.arange(len(hist)), k]
    masked = hist.copy()
    for d in (-1, 0, 1):
        masked[np.arange(len(hist)), (k + d) % 36] = -np.inf
    h2 = masked.max(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        gap = np.where(h1 > 0, (h1 - h2) / h1, np.inf)
    return gap


def angle_diff(a, b):
    d = np.mod(a - b + math.pi, 2 * math.pi) - math.pi
    return np.abs(d)


def rel_l2(g, o):
    num = np.linalg.norm(g - o, axis=1)
    den = np.linalg.norm(o, axis=1)
    return np.where(den > 0, num / np.maximum(den, 1e-300), num)


def match_margins(d1, d2, ratio):
    """Distance of a query from the two decision boundaries of the matcher:
    the ratio test (|d1/d2 - ratio|) and the nearest-neighbour tie
    ((d2 - d1) / d1)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        m1 = np.where(np.isfinite(d2) & (d2 > 0), np.abs(d1 / d2 - ratio), np.inf)
        m2 = np.where(d1 > 0, (d2 - d1) / d1, np.where(d2 > 0, np.inf, 0.0))
    return np.minimum(m1, m2)


def oracle_features_at(img, kp, Ls, idx=None, return_hist=True):
    ws = oracle.subregion_sides(Ls)[kp["scale"]]
    x, y = kp["x"], kp["y"]
    if idx is not None:
        x, y, ws = x[idx], y[idx], ws[idx]
    th, hist = oracle.orientation(img, x, y, ws, return_hist=True)
    desc = oracle.describe(img, x, y, ws, th)
    return th, desc, hist


def multi_ambiguous(h, peak_ratio=0.8, tol=1e-5):
    """True when a decision of the secondary-orientation rule on the smoothed
    histogram h is within `tol` (relative to its maximum) of its boundary: the
    threshold, a strictness test or the order of two bins that can be peaks
    (among them the dominant tie), or when the support is flat."""
    m = h.max()
    if m <= 0.0:
        return True
    best = int(np.argmax(h))
    high = [k for k in range(36) if h[k] >= (peak_ratio - tol) * m]
    for k in high:
        if k == best:                # taken whatever its neighbours and the threshold
            continue
        if abs(h[k] - peak_ratio * m) < tol * m:
            return True
        if min(abs(h[k] - h[(k - 1) % 36]), abs(h[k] - h[(k + 1) % 36])) < tol * m:
            return True
    v = np.sort(h[high])
    return bool(np.any(np.diff(v) < tol * m))
