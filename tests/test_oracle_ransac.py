"""Pins of the oracle's RANSAC homography (Sec. 2.5, Eq. 7-8)."""
import numpy as np
import pytest

import synth
from oracle import ransac as R


def rand_h(rng):
    H = synth.similarity_h(rng.uniform(-20, 20), rng.uniform(0.8, 1.2), rng.uniform(-200, 200),
                           rng.uniform(-100, 100))
    H[2, :2] = rng.uniform(-2e-5, 2e-5, 2)     # mild projective part
    return H


@pytest.mark.parametrize("seed", range(5))
def test_dlt_recovers_exact_homography(seed):
    rng = np.random.default_rng(seed)
    H = rand_h(rng)
    pa = rng.uniform(0, 2000, (4, 2))
    pb = synth.apply_h(H, pa)
    G = R.dlt(pa, pb)
    assert np.allclose(G, H / H[2, 2], rtol=1e-9, atol=1e-9)
    pa = rng.uniform(0, 2000, (50, 2))
    G = R.dlt(pa, synth.apply_h(H, pa))
    assert np.allclose(G, H / H[2, 2], rtol=1e-9, atol=1e-9)


def test_rigid_transform_of_eq8_is_recovered():
    # Eq. 8: rotation and translation only
    H = synth.similarity_h(12.0, 1.0, 35.0, -7.0)
    pa = np.random.default_rng(1).uniform(0, 500, (30, 2))
    G = R.dlt(pa, synth.apply_h(H, pa))
    th = np.degrees(np.arctan2(G[1, 0], G[0, 0]))
    assert th == pytest.approx(12.0, abs=1e-9)
    assert G[0, 2] == pytest.approx(35.0, abs=1e-7) and G[1, 2] == pytest.approx(-7.0, abs=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_planted_inliers_among_outliers(seed):
    rng = np.random.default_rng(10 + seed)
    H = rand_h(rng)
    n_in, n_out = 60, 140
    pa = rng.uniform(0, 2000, (n_in + n_out, 2))
    pb = synth.apply_h(H, pa)
    pb[:n_in] += rng.normal(0, 0.3, (n_in, 2))
    pb[n_in:] = rng.uniform(-500, 2500, (n_out, 2))
    perm = rng.permutation(n_in + n_out)
    pa, pb = pa[perm], pb[perm]
    truth = perm < n_in
    samples = synth.ransac_samples(len(pa), 2000, np.random.default_rng(seed))
    G, mask, best = R.ransac(pa, pb, samples, 3.0)
    assert best >= 0
    assert np.array_equal(mask, truth)
    corners = np.array([[0, 0], [2000, 0], [2000, 2000], [0, 2000.0]])
    assert np.abs(synth.apply_h(G, corners) - synth.apply_h(H, corners)).max() < 1.0


def test_degenerate_samples_are_skipped():
    pa = np.array([[0, 0], [1, 1], [2, 2], [3, 3], [0, 5.0]])
    pb = pa + 1.0
    G, mask, best = R.ransac(pa, pb, np.array([[0, 1, 2, 3]]), 3.0)
    assert G is None and best == -1 and not mask.any()
    G, mask, best = R.ransac(pa, pb, np.array([[0, 1, 2, 3], [0, 1, 4, 3]]), 3.0)
    # the second sample has 0, 1, 3 collinear too
    assert G is None
    pa = np.array([[0, 0], [10, 0], [0, 10], [10, 10], [5, 3.0]])
    G, mask, best = R.ransac(pa, pa + [2.0, -1.0], np.array([[0, 1, 2, 3]]), 3.0)
    assert best == 0 and mask.all()
    assert np.allclose(G, [[1, 0, 2], [0, 1, -1], [0, 0, 1]], atol=1e-12)


def test_too_few_points():
    G, mask, best = R.ransac(np.zeros((3, 2)), np.zeros((3, 2)), np.zeros((5, 4), np.int32), 3.0)
    assert G is None and len(mask) == 3


def test_samples_from_uniforms():
    rng = np.random.default_rng(4)
    u = rng.random((500, 4, 8))
    for n in (4, 5, 9, 1000):
        S = R.samples_from_uniforms(u, n)
        ok = S[:, 0] >= 0
        assert ok.mean() > (0.5 if n < 9 else 0.99)
        v = S[ok]
        assert np.all((v >= 0) & (v < n))
        assert all(len(set(r)) == 4 for r in v.tolist())
    # without collisions every slot is its first draw, floor(u n)
    n = 10 ** 6
    S = R.samples_from_uniforms(u, n)
    assert np.array_equal(S, np.floor(u[:, :, 0] * n).astype(np.int64))
    # hand-built collisions: slot 1 repeats slot 0 twice, then takes try 2
    v = np.zeros((1, 4, 8))
    v[0, :, 0] = [0.10, 0.11, 0.5, 0.9]
    v[0, 1, 1] = 0.105
    v[0, 1, 2] = 0.7
    assert R.samples_from_uniforms(v, 10).tolist() == [[1, 7, 5, 9]]
    assert np.all(R.samples_from_uniforms(u, 3) == -1)
    # a slot with no distinct try leaves the hypothesis out
    w = np.full((1, 4, 8), 0.25)
    assert R.samples_from_uniforms(w, 10).tolist() == [[-1, -1, -1, -1]]


def test_ransac_skips_invalid_rows():
    rng = np.random.default_rng(5)
    H = np.array([[1.02, 0.03, 5.0], [-0.02, 0.98, -3.0], [1e-5, 0, 1.0]])
    pa = rng.uniform(0, 500, (60, 2))
    q = np.c_[pa, np.ones(60)] @ H.T
    pb = q[:, :2] / q[:, 2:]
    samples = np.array([[-1, -1, -1, -1], [0, 1, 2, 3]])
    Hr, mask, best = R.ransac(pa, pb, samples)
    assert best == 1 and mask.all()
    assert np.allclose(Hr, H / H[2, 2], atol=1e-9)


def shifted(H, dx, dy, deg=0.0):
    """H followed by a small rotation about the origin and a shift (px)."""
    c, s = np.cos(np.radians(deg)), np.sin(np.radians(deg))
    return np.array([[c, -s, dx], [s, c, dy], [0, 0, 1.0]]) @ H


def planted(seed, n_in=60, n_out=140, noise=0.0):
    rng = np.random.default_rng(40 + seed)
    H = rand_h(rng)
    pa = rng.uniform(0, 2000, (n_in + n_out, 2))
    pb = synth.apply_h(H, pa)
    if noise > 0:
        pb[:n_in] += rng.normal(0, noise, (n_in, 2))
    pb[n_in:] = rng.uniform(-500, 2500, (n_out, 2))
    truth = np.arange(n_in + n_out) < n_in
    return H / H[2, 2], pa, pb, truth


@pytest.mark.parametrize("seed", range(4))
def test_refine_exact_points_give_the_planted_h(seed):
    # exact inliers: one least-squares round over any >= 4 of them is H itself
    H, pa, pb, truth = planted(seed)
    start = shifted(H, 1.0, -0.5)
    G, mask, rounds = R.refine(pa, pb, start, 3.0)
    assert np.array_equal(mask, truth)
    assert np.allclose(G, H, rtol=1e-9, atol=1e-9)
    assert rounds in (1, 2)


@pytest.mark.parametrize("seed", range(4))
def test_refine_iterates_until_the_inlier_set_is_stable(seed):
    # a start 2.9 px off leaves part of the planted inliers out; the first fit
    # brings them in, so a second round is needed to see the set unchanged
    H, pa, pb, truth = planted(seed, noise=0.3)
    start = shifted(H, 2.9, 0.0)
    m0 = R.reprojection_error(start, pa, pb) < 3.0
    assert m0[truth].mean() < 0.7
    G, mask, rounds = R.refine(pa, pb, start, 3.0)
    assert rounds >= 2
    assert np.array_equal(mask, truth)
    corners = np.array([[0, 0], [2000, 0], [2000, 2000], [0, 2000.0]])
    assert np.abs(synth.apply_h(G, corners) - synth.apply_h(H, corners)).max() < 0.5
    # the result is a fixed point: one more call takes one round and keeps it
    G2, mask2, rounds2 = R.refine(pa, pb, G, 3.0)
    assert rounds2 == 1 and np.array_equal(mask2, mask)
    assert np.abs(synth.apply_h(G2, corners) - synth.apply_h(G, corners)).max() < 1e-9
    # a single round stops early, with the first fit's inliers
    G1, mask1, r1 = R.refine(pa, pb, start, 3.0, max_rounds=1)
    assert r1 == 1 and np.array_equal(mask1, R.reprojection_error(G1, pa, pb) < 3.0)


def test_refine_zero_rounds_and_too_few_inliers():
    H, pa, pb, truth = planted(0, noise=0.3)
    start = shifted(H, 1.0, 1.0)
    G, mask, rounds = R.refine(pa, pb, start, 3.0, max_rounds=0)
    assert rounds == 0 and np.array_equal(G, start)
    assert np.array_equal(mask, R.reprojection_error(start, pa, pb) < 3.0)
    far = shifted(H, 400.0, 0.0)
    G, mask, rounds = R.refine(pa, pb, far, 3.0)
    assert mask.sum() < 4 and rounds == 0 and np.array_equal(G, far)
