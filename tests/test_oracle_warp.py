"""Pins of the warp-and-blend oracle (oracle/warp.py) against closed forms."""
import math

import numpy as np
import pytest

from oracle import warp as W


def rand_img(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, (h, w), dtype=np.uint8)


def test_identity_and_integer_translation_reproduce_the_image():
    img = rand_img(50, 40, 0)
    for tx, ty in ((0, 0), (7, -3), (-12, 5)):
        G = np.array([[1.0, 0, tx], [0, 1.0, ty], [0, 0, 1.0]])
        x0, y0, w, h = W.canvas_bounds([img.shape], [G])
        assert (x0, y0, w, h) == (tx, ty, 40, 50)
        c, n, _ = W.warp_blend([img], [G], x0, y0, w, h)
        assert np.array_equal(c.reshape(50, 40), img.astype(np.float64))
        assert np.all(n == 1)


def test_canvas_bounds_of_known_corners():
    G = np.array([[1.0, 0, -5.5], [0, 1.0, 2.25], [0, 0, 1.0]])
    assert W.canvas_bounds([(8, 10)], [G]) == (-6.0, 2.0, 10, 8)
    # two images: the union of both boxes
    G2 = np.array([[2.0, 0, 30.0], [0, 2.0, -1.0], [0, 0, 1.0]])      # corners x 30..48, y -1..13
    assert W.canvas_bounds([(8, 10), (8, 10)], [G, G2]) == (-6.0, -1.0, 55, 15)


@pytest.mark.parametrize("G", [
    np.array([[1.3 * math.cos(0.35), -1.3 * math.sin(0.35), 12.0],
              [1.3 * math.sin(0.35), 1.3 * math.cos(0.35), -4.0], [0, 0, 1.0]]),
    np.array([[0.9, 0.12, 3.0], [-0.08, 1.1, 7.0], [4e-4, -2e-4, 1.0]]),
])
def test_linear_ramp_is_reproduced_at_the_preimage(G):
    """Bilinear interpolation is exact on a linear function, so the canvas at
    every covered pixel equals the ramp at q = G^-1 p (solved independently)."""
    yy, xx = np.mgrid[0:50, 0:40]
    img = (10 + 2 * xx + 3 * yy).astype(np.uint8)
    x0, y0, w, h = W.canvas_bounds([img.shape], [G])
    c, n, _ = W.warp_blend([img], [G], x0, y0, w, h)
    v, u = np.mgrid[0:h, 0:w]
    P = np.stack([u.ravel() + x0, v.ravel() + y0, np.ones(u.size)])
    Q = np.linalg.solve(G, P)
    qx, qy = Q[0] / Q[2], Q[1] / Q[2]
    cov = (qx >= 0) & (qx <= 39) & (qy >= 0) & (qy <= 49)
    far = np.minimum(np.minimum(np.abs(qx), np.abs(qx - 39)), np.minimum(np.abs(qy), np.abs(qy - 49))) > 1e-9
    assert np.array_equal(n[far] == 1, cov[far])
    sel = cov & far
    assert sel.sum() > 1000
    assert np.allclose(c[sel], 10 + 2 * qx[sel] + 3 * qy[sel], atol=1e-9)
    assert np.all(c[~cov & far] == 0)


def test_two_constant_images_blend_to_the_feathered_mean():
    A = np.full((20, 30), 100, np.uint8)
    B = np.full((20, 30), 200, np.uint8)
    GA = np.eye(3)
    GB = np.array([[1.0, 0, 10.0], [0, 1.0, 5.0], [0, 0, 1.0]])
    x0, y0, w, h = W.canvas_bounds([A.shape, B.shape], [GA, GB])
    assert (x0, y0, w, h) == (0.0, 0.0, 40, 25)
    c, n, _ = W.warp_blend([A, B], [GA, GB], x0, y0, w, h)
    c, n = c.reshape(h, w), n.reshape(h, w)
    for py in range(h):
        for px in range(w):
            inA = px <= 29 and py <= 19
            inB = 10 <= px <= 39 and 5 <= py <= 24
            assert n[py, px] == inA + inB
            wa = min(px + 1, 30 - px, py + 1, 20 - py) if inA else 0
            bx, by = px - 10, py - 5
            wb = min(bx + 1, 30 - bx, by + 1, 20 - by) if inB else 0
            want = (100 * wa + 200 * wb) / (wa + wb) if wa + wb else 0.0
            assert c[py, px] == pytest.approx(want, abs=1e-12)


def test_sampled_pixels_equal_the_full_canvas():
    imgs = [rand_img(30, 45, 1), rand_img(40, 25, 2)]
    G = [np.eye(3), np.array([[0.8, -0.3, 20.0], [0.3, 0.8, 4.0], [1e-3, 0, 1.0]])]
    x0, y0, w, h = W.canvas_bounds([i.shape for i in imgs], G)
    c, n, _ = W.warp_blend(imgs, G, x0, y0, w, h)
    rng = np.random.default_rng(3)
    u = rng.integers(0, w, 300)
    v = rng.integers(0, h, 300)
    cs, ns, _ = W.warp_blend(imgs, G, x0, y0, w, h, u, v)
    assert np.array_equal(cs, c.reshape(h, w)[v, u])
    assert np.array_equal(ns, n.reshape(h, w)[v, u])
