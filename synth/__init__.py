"""Seeded synthetic inputs for LP-SIFT: textures, image pairs with a known
homography, tile sets, mixed-size image sets and random descriptor sets.

This module draws random numbers and renders images. It holds none of the
feature method's arithmetic (no extrema, gradients, histograms or distances),
so both the FP64 oracle tests and the GPU path can take their inputs from it.

Recipe (all sizes are width x height, x = column, y = row):
  texture  T(x, y) = 128 + sum_b A_b exp(-1/2 q^T S_b^-1 q), q = (x, y) - c_b,
           A_b ~ U(-80, 80), S_b = R(phi_b) diag(sx^2, sy^2) R(phi_b)^T,
           sx, sy ~ U(2, 20) px, phi_b ~ U(0, pi), c_b uniform on the canvas;
           each blob is evaluated inside +-4 max(sx, sy) of its centre.
  image A  = round_half_even(T + N(0, 2^2)), clipped to 0..255.
  image B  = round_half_even(bilinear(T, H^-1 x') + N(0, 2^2)), clipped, where
           H maps A pixel coordinates to B pixel coordinates.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 240508578


def seed_for(cfg: int, instance: int = 0) -> int:
    return SEED_BASE + 1000 * cfg + instance


# --------------------------------------------------------------------------
# geometry helpers (input generation only)
# --------------------------------------------------------------------------

def similarity_h(theta_deg: float, scale: float, tx: float, ty: float,
                 cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    """3x3 matrix x' = s R(theta) (x - c) + c + t (rotation about c)."""
    t = math.radians(theta_deg)
    c, s = math.cos(t) * scale, math.sin(t) * scale
    R = np.array([[c, -s], [s, c]])
    off = np.array([cx, cy]) - R @ np.array([cx, cy]) + np.array([tx, ty])
    H = np.eye(3)
    H[:2, :2] = R
    H[:2, 2] = off
    return H


def apply_h(H: np.ndarray, pts: np.ndarray) -> np.ndarray:
    p = np.c_[pts, np.ones(len(pts))] @ H.T
    return p[:, :2] / p[:, 2:3]


def rect_corners(w: float, h: float) -> np.ndarray:
    return np.array([[0.0, 0.0], [w - 1, 0.0], [w - 1, h - 1], [0.0, h - 1]])


def _poly_area(p: np.ndarray) -> float:
    x, y = p[:, 0], p[:, 1]
    return 0.5 * abs(float(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1))))


def _clip_poly(subject: np.ndarray, clip: np.ndarray) -> np.ndarray:
    """Sutherland-Hodgman clip of a polygon by a convex polygon (CCW or CW)."""
    def orient(poly):
        return np.sign(sum(poly[i, 0] * poly[(i + 1) % len(poly), 1]
                           - poly[(i + 1) % len(poly), 0] * poly[i, 1]
                           for i in range(len(poly))))
    sgn = orient(clip)
    out = list(subject)
    for i in range(len(clip)):
        a, b = clip[i], clip[(i + 1) % len(clip)]
        inp, out = out, []
        if not inp:
            break

        def inside(p):
            return sgn * ((b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])) >= 0

        def inter(p, q):
            d1 = (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
            d2 = (b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0])
            t = d1 / (d1 - d2)
            return p + t * (q - p)
        for j in range(len(inp)):
            p, q = inp[j], inp[(j + 1) % len(inp)]
            if inside(q):
                if not inside(p):
                    out.append(inter(p, q))
                out.append(q)
            elif inside(p):
                out.append(inter(p, q))
    return np.array(out) if out else np.zeros((0, 2))


def footprint_iou(H: np.ndarray, wa: int, ha: int, wb: int, hb: int) -> float:
    """IoU, in A's frame, of A's rectangle and B's rectangle mapped by H^-1."""
    A = rect_corners(wa, ha)
    B = apply_h(np.linalg.inv(H), rect_corners(wb, hb))
    I = _clip_poly(B, A)
    ai = _poly_area(I) if len(I) >= 3 else 0.0
    return ai / (_poly_area(A) + _poly_area(B) - ai)


# --------------------------------------------------------------------------
# texture rendering
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Canvas:
    x0: float          # canvas pixel (0, 0) sits at world (x0, y0)
    y0: float
    tex: np.ndarray    # float64 [h, w]


def render_texture(x0: float, y0: float, w: int, h: int, n_blobs: int,
                   rng: np.random.Generator, base: float = 128.0,
                   amp: float = 80.0, sig: Tuple[float, float] = (2.0, 20.0)) -> Canvas:
    tex = np.full((h, w), base, dtype=np.float64)
    cx = rng.uniform(0, w, n_blobs)
    cy = rng.uniform(0, h, n_blobs)
    sx = rng.uniform(sig[0], sig[1], n_blobs)
    sy = rng.uniform(sig[0], sig[1], n_blobs)
    phi = rng.uniform(0, math.pi, n_blobs)
    A = rng.uniform(-amp, amp, n_blobs)
    for b in range(n_blobs):
        r = 4.0 * max(sx[b], sy[b])
        xa, xb = max(0, int(cx[b] - r)), min(w, int(cx[b] + r) + 1)
        ya, yb = max(0, int(cy[b] - r)), min(h, int(cy[b] + r) + 1)
        if xa >= xb or ya >= yb:
            continue
        qx = np.arange(xa, xb, dtype=np.float64)[None, :] - cx[b]
        qy = np.arange(ya, yb, dtype=np.float64)[:, None] - cy[b]
        c, s = math.cos(phi[b]), math.sin(phi[b])
        # coordinates in the blob's principal frame
        p = c * qx + s * qy
        q = -s * qx + c * qy
        tex[ya:yb, xa:xb] += A[b] * np.exp(-0.5 * (p * p / sx[b] ** 2 + q * q / sy[b] ** 2))
    return Canvas(x0, y0, tex)


def bilinear(canvas: Canvas, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Sample the canvas at world coordinates (xs, ys); outside -> base 128."""
    t = canvas.tex
    h, w = t.shape
    u = xs - canvas.x0
    v = ys - canvas.y0
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    fu = u - i0
    fv = v - j0
    ok = (i0 >= 0) & (j0 >= 0) & (i0 + 1 < w) & (j0 + 1 < h)
    i0c = np.clip(i0, 0, w - 2)
    j0c = np.clip(j0, 0, h - 2)
    out = (t[j0c, i0c] * (1 - fu) * (1 - fv) + t[j0c, i0c + 1] * fu * (1 - fv)
           + t[j0c + 1, i0c] * (1 - fu) * fv + t[j0c + 1, i0c + 1] * fu * fv)
    return np.where(ok, out, 128.0)


def to_uint8(img: np.ndarray, rng: np.random.Generator, noise_sigma: float = 2.0,
             gain: float = 1.0) -> np.ndarray:
    noisy = gain * img + rng.normal(0.0, noise_sigma, img.shape)
    return np.clip(np.rint(noisy), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# image pairs (two-image configurations)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Pair:
    A: np.ndarray      # uint8 [h, w]
    B: np.ndarray      # uint8 [h, w]
    H: np.ndarray      # 3x3 float64, A pixel coords -> B pixel coords
    iou: float
    seed: int


def render_pair(w: int, h: int, H: np.ndarray, n_blobs_in_a: int,
                rng: np.random.Generator, wb: Optional[int] = None,
                hb: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    wb = w if wb is None else wb
    hb = h if hb is None else hb
    pre = apply_h(np.linalg.inv(H), rect_corners(wb, hb))
    allp = np.vstack([rect_corners(w, h), pre])
    x0 = math.floor(allp[:, 0].min()) - 2
    y0 = math.floor(allp[:, 1].min()) - 2
    x1 = math.ceil(allp[:, 0].max()) + 3
    y1 = math.ceil(allp[:, 1].max()) + 3
    cw, ch = x1 - x0, y1 - y0
    n_canvas = int(round(n_blobs_in_a * (cw * ch) / float(w * h)))
    canvas = render_texture(x0, y0, cw, ch, n_canvas, rng)
    a_float = canvas.tex[-y0:-y0 + h, -x0:-x0 + w]
    A = to_uint8(a_float, rng)
    yy, xx = np.mgrid[0:hb, 0:wb].astype(np.float64)
    src = apply_h(np.linalg.inv(H), np.c_[xx.ravel(), yy.ravel()])
    b_float = bilinear(canvas, src[:, 0], src[:, 1]).reshape(hb, wb)
    B = to_uint8(b_float, rng)
    return A, B


def make_pair_fixed(w: int = 640, h: int = 480, theta_deg: float = 8.0, scale: float = 1.1,
                    tx: float = 220.0, ty: float = 30.0, n_blobs: int = 200,
                    seed: Optional[int] = None) -> Pair:
    """Pair with a given rotation/scale/translation about the origin."""
    seed = seed_for(0) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    H = similarity_h(theta_deg, scale, tx, ty)
    A, B = render_pair(w, h, H, n_blobs, rng)
    return Pair(A, B, H, footprint_iou(H, w, h, w, h), seed)


def make_pair_random(w: int = 2600, h: int = 1600, n_blobs: int = 2000,
                     theta_range=(-15.0, 15.0), scale_range=(0.9, 1.15),
                     iou_range=(0.30, 0.50), seed: Optional[int] = None) -> Pair:
    """Pair whose homography is drawn at random, translation rejection-sampled
    until the footprint IoU falls in iou_range."""
    seed = seed_for(1) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(*theta_range)
    s = rng.uniform(*scale_range)
    for _ in range(100000):
        tx = rng.uniform(-w, w)
        ty = rng.uniform(-h, h)
        H = similarity_h(theta, s, tx, ty)
        iou = footprint_iou(H, w, h, w, h)
        if iou_range[0] <= iou <= iou_range[1]:
            break
    else:  # pragma: no cover
        raise RuntimeError("no translation met the overlap range")
    A, B = render_pair(w, h, H, n_blobs, rng)
    return Pair(A, B, H, iou, seed)


def config_pair(cfg: int, instance: int = 0) -> Pair:
    """The two-image workloads: 0 = 640x480 with a fixed homography,
    1 = 2600x1600 with a random one."""
    if cfg == 0:
        return make_pair_fixed(seed=seed_for(0, instance))
    if cfg == 1:
        return make_pair_random(seed=seed_for(1, instance))
    raise ValueError(cfg)


# --------------------------------------------------------------------------
# tile sets (all-pairs workload) and mixed-size image sets
# --------------------------------------------------------------------------

@dataclasses.dataclass
class TileSet:
    images: List[np.ndarray]     # uint8, in shuffled order
    H_world: List[np.ndarray]    # world -> tile pixel coordinates, same order
    order: np.ndarray            # order[k] = grid index (row-major 3x3) of image k
    seed: int


def make_tiles(world_w: int = 7000, world_h: int = 4500, grid: int = 3,
               blob_density: float = 2000 / (2600 * 1600), seed: Optional[int] = None,
               tile_w=(2600, 2800), tile_h=(1600, 1800), overlap=(0.25, 0.35),
               theta_range=(-15.0, 15.0), scale_range=(0.9, 1.15),
               gain_range=(0.9, 1.1)) -> TileSet:
    """Tiles cut from one synthetic world texture on a grid x grid layout.
    Each tile sees the world through its own similarity about its centre and
    its own gain; the set is shuffled."""
    seed = seed_for(2) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    n_blobs = int(round(blob_density * world_w * world_h))
    canvas = render_texture(0.0, 0.0, world_w, world_h, n_blobs, rng)
    tiles, Hs = [], []
    ws = rng.integers(tile_w[0], tile_w[1] + 1, grid)
    hs = rng.integers(tile_h[0], tile_h[1] + 1, grid)
    ovx = rng.uniform(overlap[0], overlap[1], grid - 1)
    ovy = rng.uniform(overlap[0], overlap[1], grid - 1)
    xs = [0.0]
    for i in range(1, grid):
        xs.append(xs[-1] + ws[i - 1] * (1 - ovx[i - 1]))
    ys = [0.0]
    for i in range(1, grid):
        ys.append(ys[-1] + hs[i - 1] * (1 - ovy[i - 1]))
    span_x = xs[-1] + ws[-1]
    span_y = ys[-1] + hs[-1]
    mx = (world_w - span_x) / 2.0
    my = (world_h - span_y) / 2.0
    for gy in range(grid):
        for gx in range(grid):
            w, h = int(ws[gx]), int(hs[gy])
            ox, oy = xs[gx] + mx, ys[gy] + my
            theta = rng.uniform(*theta_range) / 3.0
            s = rng.uniform(*scale_range)
            s = 1.0 + (s - 1.0) / 3.0
            # tile pixel p shows world point G^-1 p, with G = similarity about
            # the tile centre composed with the translation to the tile origin
            T = np.eye(3)
            T[:2, 2] = [-ox, -oy]
            S = similarity_h(theta, s, 0.0, 0.0, cx=w / 2.0, cy=h / 2.0)
            G = S @ T
            yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
            src = apply_h(np.linalg.inv(G), np.c_[xx.ravel(), yy.ravel()])
            img = bilinear(canvas, src[:, 0], src[:, 1]).reshape(h, w)
            gain = rng.uniform(*gain_range)
            tiles.append(to_uint8(img, rng, gain=gain))
            Hs.append(G)
    order = rng.permutation(grid * grid)
    return TileSet([tiles[k] for k in order], [Hs[k] for k in order], order, seed)


def mixed_pair_specs(n_pairs: int = 32, w_range=(1024, 4000), seed: Optional[int] = None,
                     blob_density: float = 2000 / (2600 * 1600)) -> List[Tuple[int, int, int, int]]:
    """(width, height, blobs, seed) of each mixed-size pair, height =
    round(0.75 width), the blob density of the 2600x1600 pair."""
    seed = seed_for(4) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_pairs):
        w = int(rng.integers(w_range[0], w_range[1] + 1))
        h = int(round(0.75 * w))
        nb = int(round(blob_density * w * h))
        out.append((w, h, nb, int(rng.integers(1 << 62))))
    return out


def make_mixed_pair(spec: Tuple[int, int, int, int]) -> Pair:
    w, h, nb, s = spec
    return make_pair_random(w, h, nb, seed=s)


def make_mixed_pairs(n_pairs: int = 32, w_range=(1024, 4000), seed: Optional[int] = None,
                     blob_density: float = 2000 / (2600 * 1600)) -> List[Pair]:
    """Pairs of mixed sizes, generated like the 2600x1600 pair with the blob
    density scaled to the image area (see mixed_pair_specs)."""
    return [make_mixed_pair(s) for s in mixed_pair_specs(n_pairs, w_range, seed, blob_density)]


# --------------------------------------------------------------------------
# descriptor sets and hypothesis samples
# --------------------------------------------------------------------------

def random_unit_rows(n: int, dim: int, rng: np.random.Generator,
                     nonneg: bool = True) -> np.ndarray:
    x = rng.random((n, dim)) if nonneg else rng.normal(size=(n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def noisy_copies(base: np.ndarray, idx: np.ndarray, sigma: float,
                 rng: np.random.Generator) -> np.ndarray:
    y = base[idx] + rng.normal(0.0, sigma, (len(idx), base.shape[1]))
    y = np.abs(y)
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    return y


def ransac_samples(n_points: int, n_iter: int, rng: np.random.Generator) -> np.ndarray:
    """n_iter x 4 distinct indices in [0, n_points), drawn once so that every
    implementation of the sampling loop sees the same hypotheses."""
    out = np.empty((n_iter, 4), dtype=np.int32)
    for i in range(n_iter):
        out[i] = rng.choice(n_points, 4, replace=False)
    return out


def scorer_init(rng: np.random.Generator, n_in: int = 258, n_hid: int = 64) -> np.ndarray:
    """Seeded starting weights of the keypoint scorer as one flat float64
    vector in the order W1 [n_hid][n_in], b1, W2 [n_hid][n_hid], b2, w3, b3:
    weights uniform in +-sqrt(6 / fan_in), biases zero."""
    parts = []
    for fan_in, shape in ((n_in, (n_hid, n_in)), (0, (n_hid,)), (n_hid, (n_hid, n_hid)),
                          (0, (n_hid,)), (n_hid, (n_hid,)), (0, (1,))):
        if fan_in == 0:
            parts.append(np.zeros(int(np.prod(shape))))
        else:
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, int(np.prod(shape))))
    return np.concatenate(parts)


def ransac_uniforms(n_iter: int, rng: np.random.Generator, tries: int = 8) -> np.ndarray:
    """[n_iter, 4, tries] uniform draws in [0, 1) from which RANSAC hypotheses
    are formed once the number of matches is known (the method's random
    draws, passed in as inputs)."""
    return rng.random((n_iter, 4, tries))
