"""FP64 oracle of multi-orientation keypoints.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The descriptor of Sec. 2.3 follows Lowe's SIFT [33], whose orientation
assignment also keeps the secondary peaks of the orientation histogram: every
other local maximum within a fixed fraction (0.8) of the highest gives the
keypoint one more orientation and one more descriptor. Reading taken here,
on the smoothed 36-bin histogram of the single-orientation oracle:
  * the dominant orientation (highest bin, lowest bin on ties, parabolic
    peak) comes first, exactly as the single-orientation oracle gives it;
  * further orientations: bins k other than the dominant one with
    sm[k] > sm[k - 1] and sm[k] > sm[k + 1] (circular, strict) and
    sm[k] >= peak_ratio * sm[dominant], highest first (lowest bin on equal
    heights), at most max_orient - 1 of them; each is refined by the parabola
    through its own bin and its two neighbours, angle (k + offset) * 10 deg;
  * every (keypoint, orientation) gives one descriptor row, keypoints in
    order, orientations in the order above.
Pins (tests/test_oracle_multi_orient.py): histogram closed forms (threshold
at exactly peak_ratio, plateaus, neighbours of the dominant bin, circular
wrap, truncation order), an image with two gradient directions of equal
weight whose orientations are exactly {0, 90} degrees, and rot90
equivariance of the orientation sets.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

import oracle as O


def peaks_from_hist(sm: np.ndarray, peak_ratio: float = 0.8, max_orient: int = 4) -> List[List[float]]:
    """Orientations (radians) of each smoothed histogram row [n][36]."""
    sm = np.asarray(sm, np.float64)
    out = []
    for h in sm:
        best = int(np.argmax(h))                 # first maximum = lowest bin on ties
        thetas = [_parabola(h, best)]
        cand = []
        for k in range(36):
            if k == best:
                continue
            if h[k] > h[(k - 1) % 36] and h[k] > h[(k + 1) % 36] and h[k] >= peak_ratio * h[best]:
                cand.append(k)
        cand.sort(key=lambda k: (-h[k], k))
        thetas += [_parabola(h, k) for k in cand[:max_orient - 1]]
        out.append(thetas)
    return out


def _parabola(h: np.ndarray, k: int) -> float:
    hm, h0, hp = h[(k - 1) % 36], h[k], h[(k + 1) % 36]
    den = hm - 2.0 * h0 + hp
    off = 0.5 * (hm - hp) / den if den != 0.0 else 0.0
    return (k + off) * 10.0 * math.pi / 180.0


def orientations(img: np.ndarray, x, y, ws, peak_ratio: float = 0.8,
                 max_orient: int = 4) -> List[List[float]]:
    """Orientation list of every keypoint; the first entry is the
    single-orientation oracle's theta0 itself."""
    th0, hist = O.orientation(img, x, y, ws, return_hist=True)
    lists = peaks_from_hist(hist, peak_ratio, max_orient)
    for t, l in zip(th0, lists):
        l[0] = float(t)
    return lists


def features_multi(img: np.ndarray, Ls, peak_ratio: float = 0.8, max_orient: int = 4,
                   d: int = 4) -> Dict[str, np.ndarray]:
    """Detect, then one descriptor row per (keypoint, orientation): rows
    (keypoint slot of each row), theta, desc, and the smoothed histograms."""
    kp = O.detect(img, Ls)
    ws = O.subregion_sides(Ls, d)[kp["scale"]]
    th0, hist = O.orientation(img, kp["x"], kp["y"], ws, return_hist=True)
    lists = peaks_from_hist(hist, peak_ratio, max_orient)
    for t, l in zip(th0, lists):
        l[0] = float(t)
    rows = np.repeat(np.arange(len(lists)), [len(l) for l in lists]).astype(np.int64)
    theta = np.array([t for l in lists for t in l], np.float64)
    desc = O.describe(img, kp["x"][rows], kp["y"][rows], ws[rows], theta, d)
    return {"kp": kp, "rows": rows, "theta": theta, "desc": desc, "hist": hist,
            "counts": np.array([len(l) for l in lists], np.int64)}
