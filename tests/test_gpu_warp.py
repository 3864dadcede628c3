"""Warp and blend on the GPU (lpsift_warp_blend) against the FP64 oracle
(oracle/warp.py).

Rules: identity and integer translations reproduce the image bit for bit;
elsewhere every canvas value is within 1e-3 of the oracle's and every count
equal, except pixels where some image's coverage decision is within 1e-6 px of
its boundary (the GPU inverts the transforms by the adjugate, the oracle by
LAPACK, so mapped points differ by rounding); those must stay rare."""
import math

import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from paper_2405_08578_amd import mosaic
from oracle import warp as W
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-3


def texture(h, w, seed, n_blobs):
    rng = np.random.Generator(np.random.PCG64(seed))
    cv = synth.render_texture(0, 0, w, h, n_blobs, rng)
    return synth.to_uint8(cv.tex, rng)


def run(gpu, imgs, G, bounds=None):
    import torch
    x0, y0, w, h = bounds or mosaic.canvas_bounds([i.shape for i in imgs], G)
    c, n = lp.warp_blend([to_dev(i, gpu) for i in imgs], G, x0, y0, w, h)
    torch.cuda.synchronize()
    return (x0, y0, w, h), c.cpu().numpy(), n.cpu().numpy()


def compare(imgs, G, b, c, n, u=None, v=None, max_near=1e-3):
    x0, y0, w, h = b
    if u is None:
        co, no, qs = W.warp_blend(imgs, G, x0, y0, w, h)
        gc, gn = c.ravel(), n.ravel()
    else:
        co, no, qs = W.warp_blend(imgs, G, x0, y0, w, h, u, v)
        gc, gn = c[v, u], n[v, u]
    near = W.near_boundary(imgs, qs)
    assert near.mean() <= max_near
    ok = ~near
    assert np.array_equal(gn[ok].astype(np.int64), no[ok])
    err = np.abs(gc[ok].astype(np.float64) - co[ok])
    assert err.max() <= TOL, f"max err {err.max()}"
    return int(ok.sum())


def test_identity_and_translation_exact(gpu):
    img = texture(97, 131, 0, 40)
    for tx, ty in ((0, 0), (17, -9)):
        G = [np.array([[1.0, 0, tx], [0, 1.0, ty], [0, 0, 1.0]])]
        say("warp identity/translation", tx, ty)
        b, c, n = run(gpu, [img], G)
        assert b == (tx, ty, 131, 97)
        assert np.array_equal(c, img.astype(np.float32))
        assert np.all(n == 1)


def test_three_images_full_canvas(gpu):
    imgs = [texture(150, 200, 1, 60), texture(180, 160, 2, 60), texture(120, 221, 3, 60)]
    G = [np.eye(3),
         np.array([[1.1 * math.cos(0.3), -1.1 * math.sin(0.3), 120.0],
                   [1.1 * math.sin(0.3), 1.1 * math.cos(0.3), 30.0], [0, 0, 1.0]]),
         np.array([[0.95, 0.1, -60.0], [-0.05, 1.05, 90.0], [3e-4, -2e-4, 1.0]])]
    say("warp three images")
    b, c, n = run(gpu, imgs, G)
    # image 0 sits on the canvas grid: its border rows and columns are flagged
    compare(imgs, G, b, c, n, max_near=0.01)
    assert n.max() == 3 and (n > 0).mean() > 0.5


def test_canvas_offset_and_partial_coverage(gpu):
    """A canvas that cuts through the images (some fully outside it) and a
    width that is not a multiple of the 4-pixel thread groups."""
    imgs = [texture(64, 80, 4, 20), texture(70, 70, 5, 20)]
    G = [np.eye(3), np.array([[0.7, -0.7, 200.0], [0.7, 0.7, 0.0], [0, 0, 1.0]])]
    say("warp partial canvas")
    b = (23.0, -11.0, 131, 77)
    _, c, n = run(gpu, imgs, G, b)
    compare(imgs, G, b, c, n, max_near=0.03)


def test_sixteen_images(gpu):
    rng = np.random.default_rng(6)
    imgs = [texture(int(rng.integers(20, 60)), int(rng.integers(20, 60)), 10 + k, 8)
            for k in range(16)]
    G = []
    for k in range(16):
        a = rng.uniform(-0.4, 0.4)
        s = rng.uniform(0.8, 1.3)
        G.append(np.array([[s * math.cos(a), -s * math.sin(a), 15.0 * (k % 4)],
                           [s * math.sin(a), s * math.cos(a), 12.0 * (k // 4)],
                           [rng.normal(0, 1e-4), rng.normal(0, 1e-4), 1.0]]))
    say("warp sixteen images")
    b, c, n = run(gpu, imgs, G)
    compare(imgs, G, b, c, n, max_near=2e-3)
    assert n.max() >= 4


def test_nine_tiles_sampled(gpu):
    """The 9-tile set with the generator's transforms composed into the frame
    of tile 0 (a canvas of about 6950 x 4430); 300,000 sampled pixels against
    the oracle; overlaps (count >= 2) must cover a large share."""
    tiles = synth.make_tiles()
    ref = 0
    G = [tiles.H_world[ref] @ np.linalg.inv(tiles.H_world[k]) for k in range(9)]
    say("warp nine tiles")
    b, c, n = run(gpu, tiles.images, G)
    x0, y0, w, h = b
    assert 6000 < w < 8000 and 4000 < h < 5000
    rng = np.random.default_rng(7)
    u = rng.integers(0, w, 300000)
    v = rng.integers(0, h, 300000)
    compare(tiles.images, G, b, c, n, u, v, max_near=2e-3)
    assert (n >= 2).mean() > 0.2


def test_without_count_buffer(gpu):
    """count may be null: the canvas is the same as with it."""
    import torch
    imgs = [texture(90, 120, 21, 30), texture(100, 80, 22, 30)]
    G = [np.eye(3), np.array([[0.9, 0.2, 60.0], [-0.2, 0.9, 30.0], [0, 0, 1.0]])]
    b = mosaic.canvas_bounds([i.shape for i in imgs], G)
    dev = [to_dev(i, gpu) for i in imgs]
    say("warp without count")
    c1, n1 = lp.warp_blend(dev, G, *b)
    c2, n2 = lp.warp_blend(dev, G, *b, with_count=False)
    torch.cuda.synchronize()
    assert n2 is None
    assert torch.equal(c1, c2)
