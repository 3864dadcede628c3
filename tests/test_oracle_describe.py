"""Pins of the oracle's orientation and descriptor (Sec. 2.3, Eq. 3-5).

Checked against closed forms of constant-gradient ramps (where the gradient
direction, the orientation bin and the spatial weights are known exactly),
a separable 1-D evaluation of the spatial binning, the 90-degree rotation
equivariance of the whole construction, gain invariance and the norm.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def ramp(gx, gy, n=64, c0=128):
    yy, xx = np.mgrid[0:n, 0:n]
    img = c0 + gx * (xx - n // 2) + gy * (yy - n // 2)
    assert img.min() >= 0 and img.max() <= 255
    return img.astype(np.uint8)


def test_subregion_sides_default_beta0():
    # w_s = sqrt(Lmin * L) / d with the largest admissible beta0 (Eq. 3-4)
    ws = oracle.subregion_sides([16, 32, 64, 128])
    assert np.allclose(ws, [4.0, math.sqrt(32), 8.0, math.sqrt(128)], rtol=1e-14)
    ws = oracle.subregion_sides([32, 40], d=4)
    assert np.allclose(ws, [8.0, math.sqrt(32 * 40) / 4], rtol=1e-14)
    # w = d w_s never exceeds L
    for Ls in ([16, 32, 64, 128], [32, 40], [100, 128], [256, 512]):
        assert np.all(4 * oracle.subregion_sides(Ls) <= np.array(Ls) * (1 + 1e-12))


def test_gradient_convention():
    img = ramp(1, 0)
    m, a = oracle.gradient_at(img, 10, 10)
    assert (m, a) == (2.0, 0.0)              # column difference b = 2, angle 0
    img = ramp(0, 1)
    m, a = oracle.gradient_at(img, 10, 10)
    assert m == 2.0 and a == pytest.approx(math.pi / 2, abs=1e-15)  # rows grow downwards


@pytest.mark.parametrize("gx,gy,deg", [(1, 0, 0.0), (0, 1, 90.0), (-1, 0, 180.0),
                                       (0, -1, 270.0), (1, 1, 45.0), (-1, 1, 135.0)])
@pytest.mark.parametrize("ws", [4.0, math.sqrt(32), 8.0])
def test_orientation_of_ramps(gx, gy, deg, ws):
    img = ramp(gx, gy)
    th = oracle.orientation(img, [32], [32], [ws])[0]
    got = math.degrees(th) % 360.0
    assert min(abs(got - deg), 360 - abs(got - deg)) < 1e-9


def test_orientation_two_bin_spike_closed_form():
    # gradient angle between bin centres: the raw histogram is a two-bin spike
    img = ramp(2, 1)
    th, hist = oracle.orientation(img, [32], [32], [4.0], return_hist=True)
    phi = math.degrees(math.atan2(2, 4))
    k0, fr = int(phi // 10), phi / 10 - int(phi // 10)
    raw = np.zeros(36)
    raw[k0], raw[k0 + 1] = 1 - fr, fr
    kern = np.array([1, 4, 6, 4, 1]) / 16
    sm = np.array([sum(kern[j] * raw[(b + j - 2) % 36] for j in range(5)) for b in range(36)])
    sm *= hist[0].sum() / sm.sum()
    assert np.allclose(hist[0], sm, rtol=1e-12, atol=1e-12)
    k = int(np.argmax(sm))
    # vertex of the parabola through the three samples around the peak
    ys = sm[[k - 1, k, k + 1]]
    A = np.vander([-1.0, 0.0, 1.0], 3)
    a2, a1, _ = np.linalg.solve(A, ys)
    assert math.degrees(th[0]) == pytest.approx((k - a1 / (2 * a2)) * 10, abs=1e-9)


def roof(g_right, g_left, x0, n=96, c0=40):
    """I = c0 + g_right (x - x0) right of column x0 and c0 + g_left (x0 - x)
    left of it: central differences give magnitude 2 g_right at angle 0
    (bin 0) for x > x0, 2 g_left at angle 180 degrees (bin 18) for x < x0,
    and |g_right - g_left| at x = x0 (bin 0 or 18 by its sign)."""
    xx = np.arange(n)
    row = np.where(xx >= x0, c0 + g_right * (xx - x0), c0 + g_left * (x0 - xx))
    img = np.tile(row, (n, 1))
    assert img.min() >= 0 and img.max() <= 255
    return img.astype(np.uint8)


def disc_column_mass(dx, R, sigma):
    """Sum over the integer offsets (dx, dy) of the disc dx^2 + dy^2 <= R^2 of
    exp(-(dx^2 + dy^2) / (2 sigma^2)): one column of the Gaussian disc."""
    if dx * dx > R * R:
        return 0.0
    h = math.isqrt(R * R - dx * dx)
    dy = np.arange(-h, h + 1)
    return float(np.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma)).sum())


def roof_histogram(ws, delta, g_right, g_left, sigma=None, R=None):
    """Smoothed 36-bin orientation histogram of the roof image at a keypoint
    delta columns right of the ridge, from geometry alone: each disc column
    votes its Gaussian mass times its gradient magnitude into bin 0 or 18.
    Default reading: sigma = w_s / 2, disc radius round(1.5 w_s)."""
    sigma = 0.5 * ws if sigma is None else sigma
    R = int(math.floor(1.5 * ws + 0.5)) if R is None else R
    raw = np.zeros(36)
    for dx in range(-R, R + 1):
        col = delta + dx                 # column relative to the ridge
        if col > 0:
            mag, b = 2.0 * g_right, 0
        elif col < 0:
            mag, b = 2.0 * g_left, 18
        else:
            mag, b = abs(g_right - g_left), (0 if g_right > g_left else 18)
        raw[b] += mag * disc_column_mass(dx, R, sigma)
    kern = np.array([1, 4, 6, 4, 1]) / 16
    return np.array([sum(kern[j] * raw[(b + j - 2) % 36] for j in range(5)) for b in range(36)])


@pytest.mark.parametrize("ws", [4.0, math.sqrt(32), 8.0, math.sqrt(128)])
@pytest.mark.parametrize("delta", [0, 1, 3, 6])
def test_orientation_spatial_weighting_absolute(ws, delta):
    """The histogram's absolute bin masses pin the Gaussian width (sigma_o =
    w_s / 2) and the disc radius (round(1.5 w_s)) of the orientation step: a
    roof image splits the disc at a known column, and the two bins receive
    the Gaussian mass of their part of the disc. A width or radius one step
    off changes the masses far beyond rounding (checked below)."""
    x0, ky = 48, 48
    img = roof(1, 3, x0)
    th, hist = oracle.orientation(img, [x0 + delta], [ky], [ws], return_hist=True)
    want = roof_histogram(ws, delta, 1, 3)
    assert np.allclose(hist[0], want, rtol=1e-12, atol=1e-12)
    # theta0: the heavier of the two symmetric peaks, exactly at its bin centre
    if abs(want[0] - want[18]) > 1e-9 * want.max():
        exp_deg = 0.0 if want[0] > want[18] else 180.0
        got = math.degrees(th[0]) % 360.0
        assert min(abs(got - exp_deg), 360 - abs(got - exp_deg)) < 1e-9
    # the pin separates the reading from nearby alternatives
    R = int(math.floor(1.5 * ws + 0.5))
    for alt in (roof_histogram(ws, delta, 1, 3, sigma=ws), roof_histogram(ws, delta, 1, 3,
                sigma=ws / 3), roof_histogram(ws, delta, 1, 3, R=R - 1),
                roof_histogram(ws, delta, 1, 3, R=R + 1)):
        assert np.max(np.abs(alt - want)) > 1e-4 * want.max()


def test_orientation_spatial_weighting_decides_theta():
    """With the keypoint right of the ridge and the steeper side on the left,
    which side wins depends on how fast the Gaussian falls off: at w_s = 8
    (sigma 4, radius 12) the left side's larger gradient outweighs its smaller
    area for small offsets and loses for larger ones. The switch offset from
    geometry alone must equal the oracle's."""
    ws = 8.0
    x0 = 48
    img = roof(1, 3, x0)
    switch = None
    for delta in range(0, 12):
        want = roof_histogram(ws, delta, 1, 3)
        th = oracle.orientation(img, [x0 + delta], [48], [ws])[0]
        side = 0.0 if want[0] > want[18] else 180.0
        got = math.degrees(th) % 360.0
        assert min(abs(got - side), 360 - abs(got - side)) < 1e-9, delta
        if side == 0.0 and switch is None:
            switch = delta
    assert switch is not None and switch > 0
    # a wider Gaussian (sigma = w_s) would move the switch
    alt = next(d for d in range(0, 12) if (lambda h: h[0] > h[18])(
        roof_histogram(ws, d, 1, 3, sigma=ws)))
    assert alt != switch


def separable_spatial(ws, d=4):
    """Per-axis sums of Gaussian x triangle weights: for theta0 = 0 and a
    constant gradient the descriptor mass of cell (cy, cx) is S[cy] S[cx]."""
    R = int(math.floor(ws * (d + 1) / 2 * math.sqrt(2)))
    offs = np.arange(-R, R + 1)
    u = offs / ws
    g = np.exp(-u * u / (2 * (d / 2) ** 2))
    S = np.array([np.sum(g * np.clip(1 - np.abs(u + (d - 1) / 2 - c), 0, None)) for c in range(d)])
    return S


def normalise(D):
    D = D / max(np.linalg.norm(D), 1e-12)
    D = np.minimum(D, 0.2)
    return D / max(np.linalg.norm(D), 1e-12)


@pytest.mark.parametrize("ws", [4.0, 8.0, math.sqrt(32)])
@pytest.mark.parametrize("gx,gy,theta0,bins", [
    (1, 0, 0.0, {0: 1.0}),
    (1, 1, 0.0, {1: 1.0}),
    (0, 1, 0.0, {2: 1.0}),
    (-1, 0, 0.0, {4: 1.0}),
    (0, 1, math.pi / 2, {0: 1.0}),
    (2, 1, 0.0, None),                 # split between direction bins 0 and 1
])
def test_descriptor_closed_form_for_ramps(ws, gx, gy, theta0, bins):
    img = ramp(gx, gy, n=80)
    D = oracle.describe(img, [40], [40], [ws], [theta0])[0].reshape(4, 4, 8)
    S = separable_spatial(ws)
    if bins is None:
        t = math.atan2(2 * gy, 2 * gx) * 8 / (2 * math.pi)
        bins = {0: 1 - t, 1: t}
    E = np.zeros((4, 4, 8))
    for o, wo in bins.items():
        E[:, :, o] = np.outer(S, S) * wo
    E = normalise(E.ravel()).reshape(4, 4, 8)
    assert np.allclose(D, E, rtol=1e-10, atol=1e-12)


def test_descriptor_cell_order_follows_columns_then_rows():
    # gradient only left of the keypoint column: right-most cell column is empty
    n = 96
    img = ramp(1, 0, n=n).astype(np.int32)
    img[:, 49:] = img[:, 48:49]
    D = oracle.describe(img.astype(np.uint8), [48], [48], [4.0], [0.0])[0].reshape(4, 4, 8)
    assert np.all(D[:, 3, :] == 0) and D[:, 0, :].sum() > 0
    # same above the keypoint row: bottom cell row (cy = 3) is empty
    img = ramp(0, 1, n=n).astype(np.int32)
    img[49:, :] = img[48:49, :]
    D = oracle.describe(img.astype(np.uint8), [48], [48], [4.0], [math.pi / 2])[0]
    # theta0 = 90 deg maps image rows onto the first descriptor axis (u = dy / ws)
    D = D.reshape(4, 4, 8)
    assert np.all(D[:, 3, :] == 0) and D[:, 0, :].sum() > 0


def texture(n=160, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    cv = synth.render_texture(0, 0, n, n, 120, rng)
    return synth.to_uint8(cv.tex, rng)


def test_rot90_equivariance():
    img = texture()
    n = img.shape[1]
    rng = np.random.default_rng(5)
    xs = rng.integers(45, 115, 24).astype(np.int32)
    ys = rng.integers(45, 115, 24).astype(np.int32)
    for ws in (4.0, math.sqrt(32), 8.0):
        th = oracle.orientation(img, xs, ys, ws)
        D = oracle.describe(img, xs, ys, ws, th)
        rot = np.ascontiguousarray(np.rot90(img))
        # np.rot90: new[i, j] = old[j, n-1-i], so old (x=c, y=r) -> new (x=r, y=n-1-c)
        xr, yr = ys.copy(), (n - 1 - xs).astype(np.int32)
        thr = oracle.orientation(rot, xr, yr, ws)
        Dr = oracle.describe(rot, xr, yr, ws, thr)
        shift = np.degrees(thr - th) % 360.0
        assert np.allclose(shift, 270.0, atol=1e-8)
        assert np.allclose(Dr, D, atol=1e-9)


def test_gain_invariance_and_norm():
    img = texture(seed=11)
    img = (img // 2).astype(np.uint8)
    rng = np.random.default_rng(9)
    xs = rng.integers(2, 158, 40).astype(np.int32)     # includes border-clipped supports
    ys = rng.integers(2, 158, 40).astype(np.int32)
    for ws in (4.0, 8.0):
        th1 = oracle.orientation(img, xs, ys, ws)
        th2 = oracle.orientation(img * 2, xs, ys, ws)
        assert np.allclose(th1, th2, atol=1e-12)
        D1 = oracle.describe(img, xs, ys, ws, th1)
        D2 = oracle.describe(img * 2, xs, ys, ws, th2)
        assert np.allclose(D1, D2, atol=1e-12)
        assert np.allclose(np.linalg.norm(D1, axis=1), 1.0, atol=1e-12)
        assert D1.min() >= 0


def test_flat_patch_gives_zero_descriptor_and_zero_orientation():
    img = np.full((40, 40), 9, np.uint8)
    th = oracle.orientation(img, [20], [20], [4.0])
    assert th[0] == 0.0
    D = oracle.describe(img, [20], [20], [4.0], th)
    assert np.all(D == 0)
