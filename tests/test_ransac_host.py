"""lpsift_ransac_host (C++ in the library, host only) against the FP64 oracle.

Same hypotheses (the sample array is an input to both), so the best hypothesis
must be the same one; the inlier masks agree except for pairs whose error lies
within 1e-6 px of the threshold; the refined homographies agree to 1e-6 px at
the image corners (both solve the same least-squares problem, the library by
normal equations, the oracle with lstsq)."""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from oracle import ransac as R


def problem(seed, n_in=80, n_out=120, noise=0.5):
    rng = np.random.default_rng(seed)
    H = synth.similarity_h(rng.uniform(-15, 15), rng.uniform(0.9, 1.15), rng.uniform(-300, 300),
                           rng.uniform(-200, 200))
    H[2, :2] = rng.uniform(-1e-5, 1e-5, 2)
    pa = rng.uniform(0, 2600, (n_in + n_out, 2))
    pb = synth.apply_h(H, pa)
    pb[:n_in] += rng.normal(0, noise, (n_in, 2))
    pb[n_in:] = rng.uniform(0, 2600, (n_out, 2))
    return pa, pb


@pytest.mark.parametrize("seed", range(8))
def test_library_matches_oracle(seed):
    pa, pb = problem(seed)
    samples = synth.ransac_samples(len(pa), 500, np.random.default_rng(100 + seed))
    Ho, mo, bo = R.ransac(pa, pb, samples, 3.0)
    Hl, ml, bl = lp.ransac(pa, pb, samples, 3.0)
    assert bl == bo
    eo = R.reprojection_error(Ho, pa, pb)
    safe = np.abs(eo - 3.0) > 1e-6
    assert np.array_equal(ml[safe], mo[safe])
    corners = np.array([[0, 0], [2600, 0], [2600, 1600], [0, 1600.0]])
    assert np.abs(synth.apply_h(Hl, corners) - synth.apply_h(Ho, corners)).max() < 1e-6


def test_degenerate_and_small_inputs():
    pa = np.array([[0, 0], [1, 1], [2, 2], [3, 3], [0, 5.0]])
    H, m, b = lp.ransac(pa, pa + 1.0, np.array([[0, 1, 2, 3]]))
    assert H is None and b == -1 and not m.any()
    H, m, b = lp.ransac(np.zeros((3, 2)), np.zeros((3, 2)), np.zeros((2, 4), np.int32))
    assert H is None and len(m) == 3
    H, m, b = lp.ransac(np.zeros((0, 2)), np.zeros((0, 2)), np.zeros((0, 4), np.int32))
    assert H is None and len(m) == 0


def test_rejects_bad_arguments():
    pa, pb = problem(1)
    with pytest.raises(lp.LpsiftError):
        lp.ransac(pa, pb, np.array([[0, 1, 2, len(pa)]]))       # index out of range
    with pytest.raises(lp.LpsiftError):
        lp.ransac(pa, pb, np.array([[0, 1, 2, 3]]), thresh=0.0)


def shifted(H, dx, dy):
    return np.array([[1, 0, dx], [0, 1, dy], [0, 0, 1.0]]) @ H


@pytest.mark.parametrize("seed", range(8))
def test_refinement_matches_oracle(seed):
    pa, pb = problem(seed)
    samples = synth.ransac_samples(len(pa), 500, np.random.default_rng(100 + seed))
    Ho, _, _ = R.ransac(pa, pb, samples, 3.0)
    corners = np.array([[0, 0], [2600, 0], [2600, 1600], [0, 1600.0]])
    for start in (Ho, shifted(Ho, 2.5, -1.0)):
        Go, mo, ro = R.refine(pa, pb, start, 3.0)
        Gl, ml, rl = lp.refine_homography(pa, pb, start, 3.0)
        assert rl == ro
        safe = np.abs(R.reprojection_error(Go, pa, pb) - 3.0) > 1e-6
        assert np.array_equal(ml[safe], mo[safe])
        assert np.abs(synth.apply_h(Gl, corners) - synth.apply_h(Go, corners)).max() < 1e-6


def test_refinement_edge_cases():
    pa, pb = problem(3)
    samples = synth.ransac_samples(len(pa), 500, np.random.default_rng(103))
    Ho, _, _ = R.ransac(pa, pb, samples, 3.0)
    G, m, r = lp.refine_homography(pa, pb, Ho, 3.0, max_rounds=0)
    assert r == 0 and np.array_equal(G, Ho)
    assert np.array_equal(m, R.reprojection_error(Ho, pa, pb) < 3.0)
    G, m, r = lp.refine_homography(pa, pb, shifted(Ho, 500.0, 0.0), 3.0)
    assert r == 0 and m.sum() < 4
    G, m, r = lp.refine_homography(np.zeros((0, 2)), np.zeros((0, 2)), np.eye(3))
    assert r == 0 and len(m) == 0
    with pytest.raises(lp.LpsiftError):
        lp.refine_homography(pa, pb, Ho, thresh=0.0)
    with pytest.raises(lp.LpsiftError):
        lp.refine_homography(pa, pb, Ho, max_rounds=-1)
    bad = Ho.copy()
    bad[0, 0] = np.nan
    with pytest.raises(lp.LpsiftError):
        lp.refine_homography(pa, pb, bad)
