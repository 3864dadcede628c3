"""Pins of the oracle's window-extremum detection (Sec. 2.1-2.2, Eq. 1-2).

Each test checks the C oracle against something computed another way:
a NumPy brute force with lexicographic sorting, Eq. 1 evaluated literally in
exact rational arithmetic, closed-form images and counting invariants.
"""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle


def brute_force(img, Ls):
    """Per window, sort pixels by (value, raster index): the last is the
    maximum, the first the minimum."""
    h, w = img.shape
    out = []
    for s, L in enumerate(Ls):
        for by in range(0, h, L):
            for bx in range(0, w, L):
                rr, cc = np.mgrid[by:min(by + L, h), bx:min(bx + L, w)]
                vals = img[rr, cc].ravel()
                ras = (rr * w + cc).ravel()
                order = np.lexsort((ras, vals))
                hi, lo = ras[order[-1]], ras[order[0]]
                out.append((hi % w, hi // w, s, +1, int(img.flat[hi])))
                out.append((lo % w, lo // w, s, -1, int(img.flat[lo])))
    return out


def as_tuples(kp):
    return list(zip(kp["x"].tolist(), kp["y"].tolist(), kp["scale"].tolist(),
                    kp["type"].tolist(), kp["value"].tolist()))


@settings(max_examples=60, deadline=None)
@given(h=st.integers(1, 40), w=st.integers(1, 40),
       Ls=st.lists(st.sampled_from([1, 2, 3, 4, 5, 8, 16]), min_size=1, max_size=3, unique=True),
       levels=st.integers(1, 256), seed=st.integers(0, 2**31))
def test_detect_matches_brute_force(h, w, Ls, levels, seed):
    rng = np.random.default_rng(seed)
    Ls = sorted(Ls)
    # few intensity levels -> many ties, which exercises the Eq. 1 tie-break
    img = rng.integers(0, levels, (h, w)).astype(np.uint8)
    kp = oracle.detect(img, Ls)
    assert as_tuples(kp) == brute_force(img, Ls)


def eq1_extrema(img, L):
    """Eq. 1 literally: M_n(i, j) = M(i, j) + ((i-1) nc + j) alpha with 1-based
    indices and alpha = 1/(nr nc + 1), in exact rationals; Eq. 2 extrema."""
    nr, nc = img.shape
    alpha = Fraction(1, nr * nc + 1)
    out = []
    for by in range(0, nr, L):
        for bx in range(0, nc, L):
            cells = []
            for r in range(by, min(by + L, nr)):
                for c in range(bx, min(bx + L, nc)):
                    i, j = r + 1, c + 1
                    cells.append((Fraction(int(img[r, c])) + ((i - 1) * nc + j) * alpha, r, c))
            mx = max(cells)
            mn = min(cells)
            out.append((mx[2], mx[1]))
            out.append((mn[2], mn[1]))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_detect_equals_eq1_in_exact_arithmetic(seed):
    rng = np.random.default_rng(100 + seed)
    h, w = rng.integers(5, 23, 2)
    img = rng.integers(0, 4, (h, w)).astype(np.uint8)   # heavy ties
    L = int(rng.choice([2, 3, 4, 7]))
    kp = oracle.detect(img, [L])
    got = list(zip(kp["x"].tolist(), kp["y"].tolist()))
    assert got == eq1_extrema(img, L)


def test_constant_image_closed_form():
    h, w, L = 37, 50, 16
    img = np.full((h, w), 77, np.uint8)
    kp = oracle.detect(img, [L])
    i = 0
    for by in range(0, h, L):
        for bx in range(0, w, L):
            r1, c1 = min(by + L, h) - 1, min(bx + L, w) - 1
            assert (kp["x"][i], kp["y"][i], kp["type"][i]) == (c1, r1, 1)   # last pixel
            assert (kp["x"][i + 1], kp["y"][i + 1], kp["type"][i + 1]) == (bx, by, -1)
            assert kp["contrast"][i] == 0.0 and kp["contrast"][i + 1] == 0.0
            i += 2


def test_raster_ramp_and_impulse():
    h, w = 15, 17                      # 255 pixels: value = raster index
    img = np.arange(h * w, dtype=np.int64).reshape(h, w).astype(np.uint8)
    kp = oracle.detect(img, [4])
    i = 0
    for by in range(0, h, 4):
        for bx in range(0, w, 4):
            assert (kp["x"][i], kp["y"][i]) == (min(bx + 4, w) - 1, min(by + 4, h) - 1)
            assert (kp["x"][i + 1], kp["y"][i + 1]) == (bx, by)
            i += 2
    imp = np.zeros((32, 32), np.uint8)
    imp[20, 9] = 255
    kp = oracle.detect(imp, [32])
    assert (kp["x"][0], kp["y"][0], kp["value"][0]) == (9, 20, 255)
    assert (kp["x"][1], kp["y"][1], kp["value"][1]) == (0, 0, 0)
    # contrast of the impulse window: |255 - 255/1024| / 255
    assert kp["contrast"][0] == pytest.approx((255 - 255 / 1024) / 255, rel=1e-15)


@pytest.mark.parametrize("h,w", [(480, 640), (1600, 2600), (1, 1), (17, 3), (100, 129)])
def test_keypoint_count(h, w):
    Ls = [16, 32, 64, 128]
    expect = sum(2 * (-(-h // L)) * (-(-w // L)) for L in Ls)
    assert oracle.num_keypoints(h, w, Ls) == expect
    if (h, w) == (480, 640):
        assert oracle.num_keypoints(h, w, [16, 32, 64]) == 3160
    if (h, w) == (1600, 2600):
        assert expect == 43396


def test_nested_windows_and_reshape_values():
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, (64, 96)).astype(np.uint8)
    kp = oracle.detect(img, [16, 32])
    n16 = 2 * 4 * 6
    key = lambda x, y: (int(img[y, x]), y * 96 + x)
    # each 32-window extremum is the best of its four 16-children
    for by in range(2):
        for bx in range(3):
            s = n16 + 2 * (by * 3 + bx)
            kids = [2 * ((2 * by + dy) * 6 + (2 * bx + dx)) for dy in (0, 1) for dx in (0, 1)]
            mx = max(kids, key=lambda k: key(kp["x"][k], kp["y"][k]))
            mn = min(kids, key=lambda k: key(kp["x"][k + 1], kp["y"][k + 1]))
            assert (kp["x"][s], kp["y"][s]) == (kp["x"][mx], kp["y"][mx])
            assert (kp["x"][s + 1], kp["y"][s + 1]) == (kp["x"][mn + 1], kp["y"][mn + 1])
    # values agree with a reshape max / min
    blocks = img.reshape(4, 16, 6, 16).transpose(0, 2, 1, 3).reshape(24, 256)
    assert np.array_equal(kp["value"][0:n16:2], blocks.max(1))
    assert np.array_equal(kp["value"][1:n16:2], blocks.min(1))


def test_contrast_two_level_window():
    img = np.zeros((4, 4), np.uint8)
    img[:, 2:] = 255
    kp = oracle.detect(img, [4])
    assert kp["contrast"][0] == pytest.approx(0.5, abs=0)
    assert kp["contrast"][1] == pytest.approx(0.5, abs=0)
