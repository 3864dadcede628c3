"""FP64 oracle of warping registered images into one canvas and blending them.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper shows stitched results (Fig. 2(f), Fig. 9, Sec. 4) without fixing
how images are composed; the reading taken here:
  * every image k has a transform G_k (3 x 3, image pixels -> reference
    pixels, as the mosaic registration returns them); canvas pixel (u, v)
    is the reference point p = (u + x0, v + y0);
  * image k covers p when q = G_k^-1 p (homogeneous, divided by its third
    coordinate) lies in [0, w_k - 1] x [0, h_k - 1];
  * its sample is the bilinear interpolation of the image at q (the
    neighbour index past the last row or column is clamped; its weight is
    zero there), its weight the distance to the image border plus one,
    min(qx + 1, w_k - qx, qy + 1, h_k - qy) (feathering);
  * canvas = sum of weight x sample / sum of weights (0 where nothing
    covers), count = number of covering images.
Pins (tests/test_oracle_warp.py): identity and integer translations
reproduce the image exactly, a linear ramp under an affine or projective map
gives the ramp at q in closed form (bilinear interpolation is exact on linear
functions), two constant images blend to the closed-form feathered mean,
coverage counts of known rectangles, and canvas bounds of known corners.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def canvas_bounds(shapes: Sequence[Tuple[int, int]], G: Sequence[np.ndarray]):
    """Smallest integer canvas covering every mapped image corner: (x0, y0,
    width, height) with x0 = floor(min x), width = floor(max x) - x0 + 1."""
    xs, ys = [], []
    for (h, w), g in zip(shapes, G):
        c = np.array([[0, 0, 1], [w - 1, 0, 1], [w - 1, h - 1, 1], [0, h - 1, 1]], np.float64)
        m = c @ np.asarray(g, np.float64).T
        xs.extend(m[:, 0] / m[:, 2])
        ys.extend(m[:, 1] / m[:, 2])
    x0, y0 = math.floor(min(xs)), math.floor(min(ys))
    return float(x0), float(y0), int(math.floor(max(xs)) - x0 + 1), int(math.floor(max(ys)) - y0 + 1)


def sample(img: np.ndarray, qx: np.ndarray, qy: np.ndarray):
    """Bilinear samples and coverage of one image at points (qx, qy)."""
    h, w = img.shape
    inside = (qx >= 0) & (qx <= w - 1) & (qy >= 0) & (qy <= h - 1)
    x = np.where(inside, qx, 0.0)
    y = np.where(inside, qy, 0.0)
    ix = np.floor(x).astype(np.int64)
    iy = np.floor(y).astype(np.int64)
    fx = x - ix
    fy = y - iy
    ix1 = np.minimum(ix + 1, w - 1)
    iy1 = np.minimum(iy + 1, h - 1)
    I = img.astype(np.float64)
    top = (1.0 - fx) * I[iy, ix] + fx * I[iy, ix1]
    bot = (1.0 - fx) * I[iy1, ix] + fx * I[iy1, ix1]
    val = (1.0 - fy) * top + fy * bot
    wgt = np.minimum(np.minimum(x + 1.0, w - x), np.minimum(y + 1.0, h - y))
    return val, wgt, inside


def map_points(Ginv: np.ndarray, px: np.ndarray, py: np.ndarray):
    X = Ginv[0, 0] * px + Ginv[0, 1] * py + Ginv[0, 2]
    Y = Ginv[1, 0] * px + Ginv[1, 1] * py + Ginv[1, 2]
    Z = Ginv[2, 0] * px + Ginv[2, 1] * py + Ginv[2, 2]
    return X / Z, Y / Z


def warp_blend(images: Sequence[np.ndarray], G: Sequence[np.ndarray], x0: float, y0: float,
               width: int, height: int, u=None, v=None):
    """Canvas values and counts at canvas pixels (u, v) (every pixel of the
    width x height canvas when u, v are None), with the mapped points of
    every image (for boundary checks)."""
    if u is None:
        v, u = np.mgrid[0:height, 0:width]
        u, v = u.ravel(), v.ravel()
    px = np.asarray(u, np.float64) + x0
    py = np.asarray(v, np.float64) + y0
    acc = np.zeros(px.shape)
    sw = np.zeros(px.shape)
    cnt = np.zeros(px.shape, np.int64)
    qs: List[Tuple[np.ndarray, np.ndarray]] = []
    for img, g in zip(images, G):
        qx, qy = map_points(np.linalg.inv(np.asarray(g, np.float64)), px, py)
        val, wgt, inside = sample(np.asarray(img), qx, qy)
        acc += np.where(inside, wgt * val, 0.0)
        sw += np.where(inside, wgt, 0.0)
        cnt += inside
        qs.append((qx, qy))
    canvas = np.where(sw > 0, acc / np.where(sw > 0, sw, 1.0), 0.0)
    return canvas, cnt, qs


def near_boundary(images: Sequence[np.ndarray], qs, margin: float = 1e-6) -> np.ndarray:
    """Pixels where some image's coverage decision is within `margin` pixels
    of its boundary, the perimeter of [0, w - 1] x [0, h - 1] (the decision may
    flip under rounding)."""
    near = None
    for img, (qx, qy) in zip(images, qs):
        h, w = np.asarray(img).shape
        in_x = (qx > -margin) & (qx < w - 1 + margin)
        in_y = (qy > -margin) & (qy < h - 1 + margin)
        dx = np.minimum(np.abs(qx), np.abs(qx - (w - 1)))
        dy = np.minimum(np.abs(qy), np.abs(qy - (h - 1)))
        n = ((dx < margin) & in_y) | ((dy < margin) & in_x)
        near = n if near is None else (near | n)
    return near
