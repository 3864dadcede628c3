"""Pins of the oracle's matcher (Sec. 2.4, Eq. 6, with the ratio test).

Checked against SciPy's k-d tree and cdist, and against hand-built sets whose
distances are exact in binary floating point.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

import oracle
import synth


@pytest.mark.parametrize("seed,nA,nB,dim", [(0, 300, 500, 128), (1, 64, 2, 16), (2, 1, 900, 128),
                                            (3, 250, 250, 8)])
def test_against_kdtree_and_cdist(seed, nA, nB, dim):
    rng = np.random.Generator(np.random.PCG64(seed))
    B = synth.random_unit_rows(nB, dim, rng)
    A = synth.noisy_copies(B, rng.integers(0, nB, nA), 0.05, rng)
    m = oracle.match(A, B, ratio=0.8)
    dd, ii = cKDTree(B).query(A, k=2)
    assert np.array_equal(m["j1"], ii[:, 0])
    assert np.allclose(m["d1"], dd[:, 0], rtol=1e-12)
    assert np.allclose(m["d2"], dd[:, 1], rtol=1e-12)
    D = cdist(A, B)
    srt = np.sort(D, axis=1)
    assert np.allclose(m["d1"], srt[:, 0], rtol=1e-12)
    assert np.allclose(m["d2"], srt[:, 1], rtol=1e-12)
    keep = srt[:, 0] < 0.8 * srt[:, 1]
    assert np.array_equal(m["match"] >= 0, keep)
    assert np.array_equal(m["match"][keep], np.argmin(D, axis=1)[keep])


def test_one_hot_distance_is_sqrt2():
    A = np.eye(4)[:1]
    B = np.eye(4)[1:]
    m = oracle.match(A, B)
    assert m["d1"][0] == math.sqrt(2) and m["d2"][0] == math.sqrt(2)
    assert m["j1"][0] == 0            # three-way tie: lowest index
    assert m["match"][0] == -1        # d1 == d2 is rejected


def test_exact_ratio_boundary():
    # d1 = 4, d2 = 5: the FP64 product 0.8 * 5 rounds to exactly 4.0, so the
    # strict test 4 < 4.0 rejects the pair
    q = np.zeros((1, 3))
    B = np.array([[4.0, 0, 0], [0, 5.0, 0]])
    m = oracle.match(q, B, ratio=0.8)
    assert (m["d1"][0], m["d2"][0], m["match"][0]) == (4.0, 5.0, -1)
    B2 = np.array([[4.0, 0, 0], [0, 5.0 + 1e-9, 0]])
    assert oracle.match(q, B2, ratio=0.8)["match"][0] == 0


def test_zero_tie_and_absolute_threshold():
    A = np.array([[1.0, 0.0]])
    B = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    m = oracle.match(A, B)
    assert (m["j1"][0], m["d1"][0], m["d2"][0], m["match"][0]) == (0, 0.0, 0.0, -1)
    B = np.array([[0.0, 1.0], [0.9, 0.0]])
    m = oracle.match(A, B, ratio=0.8)
    assert m["match"][0] == 1
    assert oracle.match(A, B, ratio=0.8, abs_thresh=0.1)["match"][0] == 1
    assert oracle.match(A, B, ratio=0.8, abs_thresh=0.1 - 1e-12)["match"][0] == -1


def test_degenerate_sizes():
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    m = oracle.match(A, np.array([[0.0, 1.0]]))
    assert list(m["j1"]) == [0, 0]
    assert np.all(np.isinf(m["d2"]))
    assert list(m["match"]) == [0, 0]          # d2 = +inf: only Delta_s can reject
    m = oracle.match(A, np.zeros((0, 2)))
    assert list(m["j1"]) == [-1, -1] and list(m["match"]) == [-1, -1]
    m = oracle.match(np.zeros((0, 2)), A)
    assert len(m["j1"]) == 0


def test_abs_threshold_only_brute_force():
    # ratio = +inf: Eq. 6's absolute threshold alone decides (no ratio test);
    # duplicated registered rows (d1 = d2) are then kept when d1 < threshold
    rng = np.random.default_rng(12)
    B = rng.normal(size=(40, 16))
    B[7] = B[3]
    A = np.vstack([B[3] + 1e-3, rng.normal(size=(25, 16))])
    tau = 4.0
    o = oracle.match(A, B, ratio=math.inf, abs_thresh=tau)
    D = cdist(A, B)
    d1 = D.min(axis=1)
    j1 = D.argmin(axis=1)
    expect = np.where(d1 < tau, j1, -1)
    assert np.array_equal(o["match"], expect)
    assert o["match"][0] == 3 and o["d1"][0] == o["d2"][0]
    # with the ratio test the same duplicate is rejected
    assert oracle.match(A, B, ratio=0.8, abs_thresh=tau)["match"][0] == -1
