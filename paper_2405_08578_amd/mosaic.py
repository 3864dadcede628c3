"""Mosaic registration of an unordered image set (Sec. 4, Fig. 8).

The pairwise homographies of all image pairs form H_M; a pair is stitchable
when its RANSAC keeps at least `min_inliers` inliers and at least `min_share`
of its matches (the paper does not say when an H_M entry is zero; on
self-similar textures many pairs that do not overlap still pass the ratio
test, and a model fitted to them keeps a small share). Rounds (reading of
Sec. 4, which leaves the joining of later references open):
  * round 1: the reference is the image with the most stitchable partners
    (lowest index on ties); it and its partners are placed, each partner with
    the transform of its pair;
  * later rounds: the next reference is the unplaced image with the most
    stitchable partners among the placed images (then the most partners
    overall, then the lowest index); it joins through its placed partner with
    the most inliers, and its unplaced partners are placed through it;
  * an unplaced image with no placed partner is left unregistered.
Transforms map image pixels to the first reference's pixels. This module is
host logic on the n x n pairwise results; the pairwise work is the GPU path
(AllPairs with RANSAC).
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np


def pair_transforms(n: int, pairs, H, inliers, matches=None, min_inliers: int = 12,
                    min_share: float = 0.05):
    """Stitchable-pair matrix from per-pair results: T[i][j] maps image i to
    image j (pair (i, j) gives H: i -> j and its inverse), W[i][j] inliers.
    A pair is stitchable when its RANSAC keeps at least min_inliers inliers
    and at least min_share of its matches (a model fitted to chance matches
    keeps few of many)."""
    T = [[None] * n for _ in range(n)]
    W = np.zeros((n, n), np.int64)
    if matches is None:
        matches = [0] * len(pairs)
    for (i, j), h, c, m in zip(pairs, H, inliers, matches):
        h = np.asarray(h, np.float64).reshape(3, 3)
        if c < min_inliers or c < min_share * m:
            continue
        if not np.all(np.isfinite(h)) or abs(np.linalg.det(h)) < 1e-12:
            continue
        T[i][j] = h / h[2, 2]
        hi = np.linalg.inv(h)
        T[j][i] = hi / hi[2, 2]
        W[i, j] = W[j, i] = int(c)
    return T, W


def register(n: int, T, W) -> Dict[str, object]:
    """Rounds of Sec. 4 over the stitchable-pair matrix; returns transforms
    (image -> reference pixels, None if unregistered), the rounds (reference
    and images placed), the placement links (image, image it was placed
    through) and the unregistered images."""
    deg = (W > 0).sum(axis=1)
    G: List[Optional[np.ndarray]] = [None] * n
    rounds = []
    if n == 0:
        return {"G": G, "rounds": rounds, "unregistered": [], "links": []}
    ref = int(np.lexsort((np.arange(n), -deg))[0])
    G[ref] = np.eye(3)
    placed = [ref]
    links = []
    for j in range(n):
        if j != ref and W[ref, j] > 0:
            G[j] = T[j][ref]
            placed.append(j)
            links.append((j, ref))
    rounds.append({"reference": ref, "placed": placed[:]})
    while True:
        left = [u for u in range(n) if G[u] is None]
        if not left:
            break
        score = [(int(sum(W[u, p] > 0 for p in range(n) if G[p] is not None)), int(deg[u]), -u)
                 for u in left]
        best = max(range(len(left)), key=lambda k: score[k])
        if score[best][0] == 0:
            break
        u = left[best]
        via = max((p for p in range(n) if G[p] is not None and W[u, p] > 0),
                  key=lambda p: (W[u, p], -p))
        G[u] = G[via] @ T[u][via]
        links.append((u, via))
        now = [u]
        for j in range(n):
            if G[j] is None and W[u, j] > 0:
                G[j] = G[u] @ T[j][u]
                now.append(j)
                links.append((j, u))
        rounds.append({"reference": u, "via": via, "placed": now})
    for k in range(n):
        if G[k] is not None:
            G[k] = G[k] / G[k][2, 2]
    return {"G": G, "rounds": rounds, "unregistered": [k for k in range(n) if G[k] is None],
            "reference": ref, "links": links}


def canvas_bounds(shapes, G):
    """Integer canvas of the registered images: (x0, y0, width, height) with
    x0 the floor of the smallest mapped corner x, width reaching the floor of
    the largest (same for y), so that canvas pixel (u, v) is reference point
    (u + x0, v + y0). shapes: (h, w) per image; G: image -> reference."""
    lo = np.array([np.inf, np.inf])
    hi = -lo
    for (h, w), g in zip(shapes, G):
        corners = np.array([[0.0, 0.0], [w - 1.0, 0.0], [w - 1.0, h - 1.0], [0.0, h - 1.0]])
        m = np.c_[corners, np.ones(4)] @ np.asarray(g, np.float64).T
        xy = m[:, :2] / m[:, 2:]
        lo = np.minimum(lo, xy.min(axis=0))
        hi = np.maximum(hi, xy.max(axis=0))
    x0, y0 = np.floor(lo)
    return float(x0), float(y0), int(np.floor(hi[0]) - x0) + 1, int(np.floor(hi[1]) - y0) + 1


def corner_error(G: np.ndarray, G_true: np.ndarray, w: int, h: int) -> float:
    """Largest distance between the image corners mapped by G and by G_true."""
    c = np.array([[0, 0, 1], [w - 1, 0, 1], [w - 1, h - 1, 1], [0, h - 1, 1]], np.float64)
    a = c @ np.asarray(G).T
    b = c @ np.asarray(G_true).T
    return float(np.max(np.linalg.norm(a[:, :2] / a[:, 2:] - b[:, :2] / b[:, 2:], axis=1)))


def seam_errors(G, G_true, shapes, step: int = 64) -> Dict[tuple, float]:
    """Alignment error of every truly overlapping pair of registered images:
    points of image i on a `step` grid that the true transforms place inside
    image j are mapped by both estimated transforms into the reference frame;
    the largest distance between the two mappings, per pair (i, j)."""
    out = {}
    n = len(G)
    for i in range(n):
        if G[i] is None:
            continue
        h, w = shapes[i]
        ys, xs = np.mgrid[0:h:step, 0:w:step]
        P = np.c_[xs.ravel(), ys.ravel(), np.ones(xs.size)].astype(np.float64)
        for j in range(n):
            if j == i or G[j] is None:
                continue
            Tij = np.linalg.inv(G_true[j]) @ G_true[i]          # true i -> j
            q = P @ Tij.T
            q = q[:, :2] / q[:, 2:]
            hj, wj = shapes[j]
            inside = (q[:, 0] >= 0) & (q[:, 0] <= wj - 1) & (q[:, 1] >= 0) & (q[:, 1] <= hj - 1)
            if inside.sum() < 4:
                continue
            a = P[inside] @ np.asarray(G[i]).T
            b = np.c_[q[inside], np.ones(inside.sum())] @ np.asarray(G[j]).T
            d = np.linalg.norm(a[:, :2] / a[:, 2:] - b[:, :2] / b[:, 2:], axis=1)
            out[(i, j)] = float(d.max())
    return out


def _map(G: np.ndarray, p: np.ndarray) -> np.ndarray:
    q = p @ G[:, :2].T + G[:, 2]
    return q[:, :2] / q[:, 2:3]


def refine(G, correspondences, reference: int, iters: int = 20, lam: float = 1e-3):
    """Joint refinement of the placed transforms (a step beyond Sec. 4, whose
    rounds chain pair homographies: errors then add up along the chain, and
    overlaps between images placed through different links do not agree).
    Every transform G_k (image k -> reference pixels, h33 = 1) except the
    reference's is adjusted to minimise the sum over all stitchable pairs
    (i, j) and their RANSAC-inlier correspondences (p_i, p_j) of
    |G_i(p_i) - G_j(p_j)|^2 in reference pixels, by Levenberg-Marquardt with
    the chained transforms as the start; the reference stays the identity.
    correspondences: list of (i, j, P_i [m, 2], P_j [m, 2]) in pixels.
    Returns (the refined transform list, {"rms_before", "rms_after", "iters"})."""
    n = len(G)
    free = [k for k in range(n) if G[k] is not None and k != reference]
    pos = {k: t for t, k in enumerate(free)}
    used = [(i, j, np.asarray(a, np.float64), np.asarray(b, np.float64))
            for i, j, a, b in correspondences
            if G[i] is not None and G[j] is not None and len(a) > 0 and (i in pos or j in pos)]
    if not free or not used:
        return [None if g is None else np.asarray(g, np.float64) for g in G], \
            {"rms_before": 0.0, "rms_after": 0.0, "iters": 0}
    # normalise pixel coordinates per image for a well-conditioned solve:
    # parameters are the 8 entries of S G_k S_k^-1 (h33 = 1), with S_k the
    # image's own scaling and S the reference frame's
    scale = 1.0 / 1000.0
    S = np.diag([scale, scale, 1.0])
    Si = np.diag([1.0 / scale, 1.0 / scale, 1.0])

    def to_params(Gs):
        x = np.empty(8 * len(free))
        for k in free:
            M = S @ Gs[k] @ Si
            M = M / M[2, 2]
            x[8 * pos[k]:8 * pos[k] + 8] = M.ravel()[:8]
        return x

    def from_params(x):
        out = [None if g is None else np.asarray(g, np.float64) for g in G]
        for k in free:
            M = np.append(x[8 * pos[k]:8 * pos[k] + 8], 1.0).reshape(3, 3)
            out[k] = Si @ M @ S
        return out

    def residuals(x):
        Gs = from_params(x)
        r = [(_map(Gs[i], a) - _map(Gs[j], b)).ravel() for i, j, a, b in used]
        return np.concatenate(r)

    x = to_params(G)
    r = residuals(x)
    rms0 = float(np.sqrt(np.mean(r ** 2)))
    cost = float(r @ r)
    it = 0
    for it in range(1, iters + 1):
        J = np.empty((r.size, x.size))
        for c in range(x.size):
            h = 1e-7 * max(1.0, abs(x[c]))
            xp = x.copy()
            xp[c] += h
            J[:, c] = (residuals(xp) - r) / h
        A = J.T @ J
        g = J.T @ r
        while True:
            step = np.linalg.solve(A + lam * np.diag(np.diag(A) + 1e-12), -g)
            xn = x + step
            rn = residuals(xn)
            cn = float(rn @ rn)
            if cn < cost:
                x, r, cost = xn, rn, cn
                lam = max(lam / 10.0, 1e-12)
                break
            lam *= 10.0
            if lam > 1e12:
                break
        if lam > 1e12 or float(np.linalg.norm(step)) < 1e-12 * (1.0 + float(np.linalg.norm(x))):
            break
    out = from_params(x)
    return out, {"rms_before": rms0, "rms_after": float(np.sqrt(np.mean(r ** 2))), "iters": it}


def correspondences(pairs, kps, slotA, slotB, inlier, stats, W):
    """RANSAC-inlier correspondences of the stitchable pairs (W[i, j] > 0) as
    (i, j, P_i, P_j) pixel arrays, from host copies of the GPU RANSAC outputs:
    per pair p the first stats[p, 0] entries of slotA[p], slotB[p], inlier[p];
    kps[k] holds the keypoint x, y arrays of image k."""
    out = []
    for p, (i, j) in enumerate(pairs):
        if W[i, j] <= 0:
            continue
        m = int(stats[p, 0])
        keep = np.asarray(inlier[p][:m]).astype(bool)
        sa = np.asarray(slotA[p][:m])[keep]
        sb = np.asarray(slotB[p][:m])[keep]
        Pi = np.stack([kps[i]["x"][sa], kps[i]["y"][sa]], axis=1).astype(np.float64)
        Pj = np.stack([kps[j]["x"][sb], kps[j]["y"][sb]], axis=1).astype(np.float64)
        out.append((i, j, Pi, Pj))
    return out
