"""FP64 oracle of the host RANSAC homography (Sec. 2.5, Eq. 7).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper fits the transformation of Eq. 7 between matched pairs with RANSAC
[50, 51] and states no iteration count, sampling or threshold. Reading (also
used by the product's lpsift_ransac_host):
  * a full homography (8 degrees of freedom, h33 = 1), so the configurations'
    scale changes are representable; the rigid form of Eq. 8 is a special case;
  * each hypothesis is the exact solution through 4 sampled pairs, in Hartley
    coordinates (centroid at 0, mean distance sqrt(2)) for A and for B;
  * hypotheses are given as an [n_iter, 4] index array (the random draws are
    inputs); a hypothesis is degenerate, and skipped, when 3 of its 4 points in
    A or in B are nearly collinear (|cross| <= 1e-6 x the squared bounding
    extent of those 4 points);
  * a pair is an inlier when the one-way reprojection error |H pA - pB| < thresh
    (points mapped behind the camera plane, |w| <= 1e-12, are outliers);
  * the best hypothesis has the most inliers (earliest on ties); H is then
    re-estimated by linear least squares (h33 = 1, Hartley coordinates) over
    its inliers, and the returned mask is the inlier set of that final H.
Refinement to a fixed point (reading, also the product's lpsift_refine_host:
the paper leaves the refinement of the winning model open): from a given H,
repeat the least-squares fit over the inliers of the current H until the fit
leaves the inlier set unchanged, fewer than 4 inliers remain, or the round
limit is reached.
Pins: exact correspondences recover H to ~1e-12; planted inliers among random
outliers are all recovered; degenerate samples are skipped; refinement from a
perturbed start recovers the planted H and exactly the planted inliers, and
its result is a fixed point (a second call changes nothing).
"""
from __future__ import annotations

import numpy as np


def hartley(p: np.ndarray):
    c = p.mean(axis=0)
    d = np.sqrt(((p - c) ** 2).sum(axis=1)).mean()
    s = np.sqrt(2.0) / d if d > 0 else 1.0
    T = np.array([[s, 0, -s * c[0]], [0, s, -s * c[1]], [0, 0, 1.0]])
    return T


def apply(H: np.ndarray, p: np.ndarray):
    q = np.c_[p, np.ones(len(p))] @ H.T
    return q[:, :2], q[:, 2]


def dlt(pa: np.ndarray, pb: np.ndarray):
    """Least-squares homography with h33 = 1 in Hartley coordinates."""
    Ta, Tb = hartley(pa), hartley(pb)
    a, _ = apply(Ta, pa)
    b, _ = apply(Tb, pb)
    n = len(a)
    M = np.zeros((2 * n, 8))
    r = np.zeros(2 * n)
    x, y, u, v = a[:, 0], a[:, 1], b[:, 0], b[:, 1]
    M[0::2, 0], M[0::2, 1], M[0::2, 2] = x, y, 1
    M[0::2, 6], M[0::2, 7] = -u * x, -u * y
    M[1::2, 3], M[1::2, 4], M[1::2, 5] = x, y, 1
    M[1::2, 6], M[1::2, 7] = -v * x, -v * y
    r[0::2], r[1::2] = u, v
    h, *_ = np.linalg.lstsq(M, r, rcond=None)
    Hn = np.append(h, 1.0).reshape(3, 3)
    H = np.linalg.inv(Tb) @ Hn @ Ta
    return H / H[2, 2]


def degenerate(p: np.ndarray) -> bool:
    ext = max(np.ptp(p[:, 0]), np.ptp(p[:, 1]))
    tol = 1e-6 * ext * ext
    for i in range(4):
        for j in range(i + 1, 4):
            for k in range(j + 1, 4):
                e1, e2 = p[j] - p[i], p[k] - p[i]
                if abs(e1[0] * e2[1] - e1[1] * e2[0]) <= tol:
                    return True
    return False


def reprojection_error(H: np.ndarray, pa: np.ndarray, pb: np.ndarray):
    q, w = apply(H, pa)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.sqrt((q[:, 0] / w - pb[:, 0]) ** 2 + (q[:, 1] / w - pb[:, 1]) ** 2)
    return np.where(np.abs(w) > 1e-12, e, np.inf)


def samples_from_uniforms(u: np.ndarray, n: int) -> np.ndarray:
    """Hypothesis indices from uniform draws u [n_iter, 4, tries] in [0, 1)
    when the number of matches n is only known at run time: slot s takes the
    first try t whose floor(u n) differs from the indices of slots < s; a
    hypothesis with a slot that finds none is -1 (skipped)."""
    u = np.asarray(u, np.float64)
    out = np.full((u.shape[0], 4), -1, np.int64)
    if n < 4:
        return out
    for it in range(u.shape[0]):
        got = []
        for s in range(4):
            for t in range(u.shape[2]):
                i = min(int(np.floor(u[it, s, t] * n)), n - 1)
                if i not in got:
                    got.append(i)
                    break
            else:
                break
        if len(got) == 4:
            out[it] = got
    return out


def ransac(pa: np.ndarray, pb: np.ndarray, samples: np.ndarray, thresh: float = 3.0):
    """Returns (H or None, inlier mask, best hypothesis index). Rows of
    samples holding -1 are skipped."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    n = len(pa)
    best, best_cnt = -1, -1
    for it, idx in enumerate(np.asarray(samples)):
        if n < 4 or np.any(idx < 0) or degenerate(pa[idx]) or degenerate(pb[idx]):
            continue
        H = dlt(pa[idx], pb[idx])
        cnt = int((reprojection_error(H, pa, pb) < thresh).sum())
        if cnt > best_cnt:
            best, best_cnt = it, cnt
    if best < 0:
        return None, np.zeros(n, bool), -1
    idx = np.asarray(samples)[best]
    H0 = dlt(pa[idx], pb[idx])
    inl = reprojection_error(H0, pa, pb) < thresh
    H = dlt(pa[inl], pb[inl]) if inl.sum() >= 4 else H0
    mask = reprojection_error(H, pa, pb) < thresh
    return H, mask, best


def refine(pa: np.ndarray, pb: np.ndarray, H: np.ndarray, thresh: float = 3.0,
           max_rounds: int = 20):
    """Least-squares rounds from H over the inliers of the current H, until
    the inlier set stops changing. Returns (H, inlier mask, rounds taken)."""
    pa = np.asarray(pa, np.float64)
    pb = np.asarray(pb, np.float64)
    H = np.asarray(H, np.float64).reshape(3, 3)
    mask = reprojection_error(H, pa, pb) < thresh
    rounds = 0
    while rounds < max_rounds and mask.sum() >= 4:
        F = dlt(pa[mask], pb[mask])
        if not np.all(np.isfinite(F)):
            break
        rounds += 1
        H = F
        new = reprojection_error(H, pa, pb) < thresh
        done = bool(np.array_equal(new, mask))
        mask = new
        if done:
            break
    return H, mask, rounds
