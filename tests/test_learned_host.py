"""The committed scorer weight file and its metadata, on the host: it loads,
its checksum matches, and a tampered or truncated copy is refused."""
import json
import os
import shutil

import numpy as np
import pytest

from paper_2405_08578_amd import learned as L


def test_committed_weights_load():
    w, info = L.load_weights(L.DEFAULT_WEIGHTS)
    assert w.numel() == 20801 and info["params"] == 20801
    assert np.all(np.isfinite(w.numpy()))
    for k in ("train_pairs", "steps", "seed", "heldout", "heldout_gt_match_retention"):
        assert k in info
    assert info["train_instances"][0] >= 100           # disjoint from the benchmark pair


def test_save_load_roundtrip_and_tamper(tmp_path):
    rng = np.random.default_rng(0)
    w = rng.normal(size=20801).astype(np.float32)
    p = str(tmp_path / "w")
    L.save_weights(p, w, {"note": "test"})
    back, info = L.load_weights(p)
    assert np.array_equal(back.numpy(), w) and info["note"] == "test"
    raw = bytearray(open(p + ".bin", "rb").read())
    raw[100] ^= 1
    open(p + ".bin", "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        L.load_weights(p)
    with pytest.raises(ValueError):
        L.save_weights(p, w[:100], {})


def test_gt_consistent_count():
    H = np.array([[1.0, 0, 5], [0, 1, -2], [0, 0, 1]])
    a = np.array([[0.0, 0], [10, 10], [3, 4]])
    b = a + [5, -2]
    b[2] += [3.5, 0]                                 # 3.5 px off
    assert L.gt_consistent(a, b, H) == 2
    assert L.gt_consistent(a[:0], b[:0], H) == 0


def test_hypothesis_samples():
    """Seeded, in range, 4 distinct indices per row, and spread over all
    indices (each of n = 10 appears in 40 +- 8 % of 20,000 rows)."""
    for n, it, seed in ((4, 10, 0), (57, 300, 5), (1000, 50, 11)):
        a = L.hypothesis_samples(n, it, seed)
        assert a.shape == (it, 4) and a.dtype == np.int32
        assert np.array_equal(a, L.hypothesis_samples(n, it, seed))
        assert a.min() >= 0 and a.max() < n
        s = np.sort(a, axis=1)
        assert np.all(s[:, 1:] != s[:, :-1])
    a = L.hypothesis_samples(10, 20000, 3)
    freq = np.bincount(a.ravel(), minlength=10) / 20000
    assert np.all(np.abs(freq - 0.4) < 0.032)


def test_inlier_retention_counts_slot_pairs():
    pl = {"inlier_slots": (np.array([1, 2, 3, 7]), np.array([10, 20, 30, 70]))}
    le = {"inlier_slots": (np.array([2, 3, 7, 9]), np.array([20, 31, 70, 90]))}
    assert L.inlier_retention(pl, le) == (2, 4)        # (2, 20) and (7, 70)
    assert L.inlier_retention({"inlier_slots": (np.array([], int), np.array([], int))}, le) == (0, 0)
    assert L.needs_fallback({"inliers": 11}) and not L.needs_fallback({"inliers": 12})
