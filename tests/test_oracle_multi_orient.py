"""Pins of the multi-orientation oracle (oracle/multi_orient.py): secondary
peaks of the smoothed orientation histogram (Lowe's rule, read as in the
module header) on histograms whose answers are known in closed form, an image
with two gradient directions of equal weight, and rot90 equivariance."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import multi_orient as MO
from gpu_util import multi_ambiguous


def bins(thetas):
    return [t * 180.0 / math.pi / 10.0 for t in thetas]


def hist_with(peaks, base=0.1):
    h = np.full(36, base)
    for k, v in peaks.items():
        h[k] = v
    return h[None, :]


def test_threshold_is_inclusive_and_strict_peaks_only():
    # 8 = 0.8 * 10 exactly in double: kept; 7.99 is not
    assert bins(MO.peaks_from_hist(hist_with({5: 10.0, 20: 8.0}))[0]) == pytest.approx([5, 20])
    assert bins(MO.peaks_from_hist(hist_with({5: 10.0, 20: 7.99}))[0]) == pytest.approx([5])
    # a plateau of two equal bins is not a strict maximum
    assert bins(MO.peaks_from_hist(hist_with({5: 10.0, 20: 9.0, 21: 9.0}))[0]) == pytest.approx([5])
    # a bin next to the dominant one is never a peak of its own
    assert bins(MO.peaks_from_hist(hist_with({5: 10.0, 6: 9.5}))[0])[:1] == pytest.approx(
        [5 + 0.5 * (0.1 - 9.5) / (0.1 - 20.0 + 9.5)])
    assert len(MO.peaks_from_hist(hist_with({5: 10.0, 6: 9.5}))[0]) == 1
    # peak_ratio 1: only equal heights survive
    assert len(MO.peaks_from_hist(hist_with({5: 10.0, 20: 9.999}), peak_ratio=1.0)[0]) == 1


def test_dominant_ties_wrap_and_truncation():
    # equal heights: the lower bin is dominant, the other follows
    assert bins(MO.peaks_from_hist(hist_with({20: 10.0, 5: 10.0}))[0]) == pytest.approx([5, 20])
    # circular neighbours: bin 35 between bins 34 and 0, bin 0 between 35 and 1
    assert bins(MO.peaks_from_hist(hist_with({18: 10.0, 35: 9.0}))[0]) == pytest.approx([18, 35])
    assert bins(MO.peaks_from_hist(hist_with({18: 10.0, 0: 9.0}))[0]) == pytest.approx([18, 0])
    # five qualifying peaks, max_orient = 4: the three highest after the
    # dominant, highest first, lower bin on equal heights
    h = hist_with({2: 10.0, 30: 9.0, 10: 9.5, 20: 8.5, 14: 9.0})
    assert bins(MO.peaks_from_hist(h)[0]) == pytest.approx([2, 10, 14, 30])
    assert bins(MO.peaks_from_hist(h, max_orient=2)[0]) == pytest.approx([2, 10])
    assert bins(MO.peaks_from_hist(h, max_orient=1)[0]) == pytest.approx([2])


def test_parabola_closed_form():
    h = hist_with({17: 10.0, 3: 6.8, 4: 8.5, 5: 5.0})
    # bin 4: neighbours 6.8 and 5.0 around 8.5 -> offset 0.5 (6.8 - 5) / (6.8 - 17 + 5)
    off = 0.5 * (6.8 - 5.0) / (6.8 - 17.0 + 5.0)
    assert bins(MO.peaks_from_hist(h)[0]) == pytest.approx([17, 4 + off])


def two_direction_image(n=64, x0=32, y0=32, s=2):
    yy, xx = np.mgrid[0:n, 0:n]
    img = 100 + s * np.maximum(xx - x0, yy - y0)
    assert img.min() >= 0 and img.max() <= 255
    return img.astype(np.uint8)


def test_two_gradient_directions_give_0_and_90_degrees():
    """I = 100 + 2 max(x - 32, y - 32): gradients point along the columns
    (0 deg) on one side of the diagonal and along the rows (90 deg) on the
    other, with mirror-equal weights; the diagonal's 45-degree votes split
    evenly into bins 4 and 5 (a plateau, not a peak). The two orientations are
    exactly 0 and 90 degrees (up to rounding in the angle conversion)."""
    img = two_direction_image()
    for ws in (4.0, 6.0, 8.0):
        l = MO.orientations(img, [32], [32], [ws])[0]
        assert len(l) == 2
        deg = sorted(np.degrees(np.array(l)) % 360.0)
        assert deg == pytest.approx([0.0, 90.0], abs=1e-9)
        # with a ratio above 1 nothing but the dominant orientation survives
        assert len(MO.orientations(img, [32], [32], [ws], peak_ratio=1.01)[0]) == 1


def texture(n=160, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    cv = synth.render_texture(0, 0, n, n, 120, rng)
    return synth.to_uint8(cv.tex, rng)


def ambiguous(h):
    return multi_ambiguous(h, 0.8, tol=1e-9)


def test_rot90_rotates_every_orientation():
    img = texture()
    n = img.shape[1]
    rng = np.random.default_rng(5)
    xs = rng.integers(45, 115, 300).astype(np.int32)
    ys = rng.integers(45, 115, 300).astype(np.int32)
    rot = np.ascontiguousarray(np.rot90(img))
    xr, yr = ys.copy(), (n - 1 - xs).astype(np.int32)     # old (x, y) -> new (y, n-1-x)
    multi = 0
    for ws in (4.0, math.sqrt(32), 8.0):
        _, hist = oracle.orientation(img, xs, ys, ws, return_hist=True)
        a = MO.orientations(img, xs, ys, ws)
        b = MO.orientations(rot, xr, yr, ws)
        for k in range(len(xs)):
            if ambiguous(hist[k]):
                continue
            assert len(a[k]) == len(b[k])
            multi += len(a[k]) > 1
            shift = (np.degrees(np.array(b[k]) - np.array(a[k]))) % 360.0
            assert np.allclose(shift, 270.0, atol=1e-8)
    assert multi >= 30          # the texture has secondary peaks to rotate


def test_features_multi_rows():
    img = texture(n=96, seed=4)
    r = MO.features_multi(img, [16, 32])
    kp, th0 = oracle.features(img, [16, 32])[:2]
    assert np.array_equal(np.bincount(r["rows"], minlength=len(kp["x"])), r["counts"])
    first = np.r_[0, np.cumsum(r["counts"])[:-1]]
    assert np.array_equal(r["theta"][first], th0)          # dominant = single orientation
    assert np.all(r["counts"] >= 1) and np.all(r["counts"] <= 4)
    assert r["counts"].sum() > len(kp["x"])
    assert np.allclose(np.linalg.norm(r["desc"], axis=1)[np.linalg.norm(r["desc"], axis=1) > 0],
                       1.0, atol=1e-12)
