"""The bound behind the fixed-point scale of the descriptor votes (Sec. 2.3,
Eq. 3-5, as accumulated by lpsift_describe): a bin takes, from every pixel
of its cell's support, at most 362 (above the largest gradient magnitude
255 sqrt 2) times the cell's bilinear weight, and over the integer pixels
these weights sum to less than w_s^2 + 4.5 w_s + 1 at any angle and cell
position; the support holds fewer than (2 sqrt 2 w_s + 2)^2 pixels (one
rounding of at most 1/2 each). Checked here by brute force over random
angles and cell centres, for the subregion sides of the default geometry and
a few others."""
import math

import numpy as np
import pytest


def bilinear_sums(ws, rng, trials):
    R = int(math.ceil(2.0 * math.sqrt(2.0) * ws)) + 3
    ys, xs = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    worst_sum, worst_n = 0.0, 0
    for _ in range(trials):
        th = rng.uniform(0.0, 2.0 * math.pi)
        c, s = math.cos(th), math.sin(th)
        cx, cy = rng.uniform(-0.5, 0.5, 2)   # sub-pixel position of the cell centre
        u = (c * (xs - cx) + s * (ys - cy)) / ws
        v = (c * (ys - cy) - s * (xs - cx)) / ws
        wgt = np.clip(1.0 - np.abs(u), 0.0, None) * np.clip(1.0 - np.abs(v), 0.0, None)
        worst_sum = max(worst_sum, wgt.sum())
        worst_n = max(worst_n, int((wgt > 0).sum()))
    return worst_sum, worst_n


def test_largest_gradient_below_362():
    assert math.hypot(255, 255) < 362


@pytest.mark.parametrize("ws", [1.0, 2.5, 4.0, 4.0 * math.sqrt(2.0), 8.0, 8.0 * math.sqrt(2.0), 23.7])
def test_cell_weight_sum_and_support_bounds(ws):
    rng = np.random.default_rng(int(ws * 1000))
    s, n = bilinear_sums(ws, rng, 400)
    assert s < ws * ws + 4.5 * ws + 1.0
    assert n < (2.0 * math.sqrt(2.0) * ws + 2.0) ** 2
    # the integral of the weights is w_s^2: the bound is not loose by much
    assert s > 0.9 * ws * ws


def test_scale_keeps_every_bin_below_2_to_32():
    # the library's scale: (0.98 2^32 - n_votes / 2) / (362 B)
    for ws in (0.5, 4.0, 11.3, 565.0):
        B = ws * ws + 4.5 * ws + 1.0
        nv = (2.0 * math.sqrt(2.0) * ws + 2.0) ** 2
        scale = np.float32((0.98 * 2.0 ** 32 - 0.5 * nv) / (362.0 * B))
        # largest bin: every vote at the largest value, rounded up by 1/2,
        # with float32 rounding of the scaled vote (relative 2^-23 per step)
        worst = float(scale) * 362.0 * B * (1.0 + 2.0 ** -20) + 0.5 * nv
        assert 0.0 < worst < 2.0 ** 32
