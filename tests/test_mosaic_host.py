"""The mosaic rounds of Sec. 4 on hand-built stitchable-pair matrices (host
logic only): reference choice, later rounds through the best placed partner,
unregistered images, and composition of transforms."""
import numpy as np

from paper_2405_08578_amd import mosaic as M


def translations(n, shifts):
    """Image i sits at shifts[i] in a common frame: pixel p of i is world p + s_i."""
    return [np.array([[1, 0, s[0]], [0, 1, s[1]], [0, 0, 1.0]]) for s in shifts]


def pairwise(W_list, world):
    n = len(world)
    pairs, H, inl = [], [], []
    for (i, j, c) in W_list:
        # H: i -> j = world_j^-1 world_i
        pairs.append((i, j))
        H.append(np.linalg.inv(world[j]) @ world[i])
        inl.append(c)
    return pairs, H, inl


def test_rounds_and_composition():
    shifts = [(0, 0), (100, 0), (200, 0), (0, 80), (300, 0), (900, 900)]
    world = translations(6, shifts)
    # chain 0-1-2-4, 0-3; image 5 has no partner; one weak pair below threshold
    pairs, H, inl = pairwise([(0, 1, 50), (1, 2, 60), (2, 4, 40), (0, 3, 30), (1, 3, 20),
                              (3, 4, 5)], world)
    T, W = M.pair_transforms(6, pairs, H, inl, min_inliers=12)
    assert W[3, 4] == 0 and W[1, 3] == 20
    r = M.register(6, T, W)
    # image 1 has the most partners (0, 2, 3)
    assert r["reference"] == 1 and r["rounds"][0]["placed"] == [1, 0, 2, 3]
    # 4 joins in round 2 through 2, the only placed partner
    assert r["rounds"][1]["reference"] == 4 and r["rounds"][1]["via"] == 2
    assert r["unregistered"] == [5]
    assert r["links"] == [(0, 1), (2, 1), (3, 1), (4, 2)]
    for k in (0, 1, 2, 3, 4):
        G_true = np.linalg.inv(world[1]) @ world[k]
        assert M.corner_error(r["G"][k], G_true, 50, 40) < 1e-9


def test_ties_and_best_partner():
    shifts = [(0, 0), (10, 0), (20, 0), (30, 0)]
    world = translations(4, shifts)
    pairs, H, inl = pairwise([(0, 1, 30), (2, 3, 30), (1, 2, 15), (0, 3, 90)], world)
    T, W = M.pair_transforms(4, pairs, H, inl)
    r = M.register(4, T, W)
    assert r["reference"] == 0                       # all have 2 partners: lowest index
    assert sorted(r["rounds"][0]["placed"]) == [0, 1, 3]
    assert r["rounds"][1]["reference"] == 2 and r["rounds"][1]["via"] == 3   # 30 inliers vs 15 via 1
    assert r["unregistered"] == []


def test_degenerate_inputs():
    r = M.register(0, [], np.zeros((0, 0), int))
    assert r["G"] == [] and r["unregistered"] == []
    T, W = M.pair_transforms(2, [(0, 1)], [np.zeros(9)], [100])
    assert W[0, 1] == 0                              # singular H is not stitchable
    r = M.register(2, T, W)
    assert r["unregistered"] == [1]


def similarity(theta_deg, s, tx, ty):
    t = np.radians(theta_deg)
    return np.array([[s * np.cos(t), -s * np.sin(t), tx], [s * np.sin(t), s * np.cos(t), ty],
                     [0, 0, 1.0]])


def test_refine_removes_chained_drift():
    """A 2 x 3 grid of 800 x 600 images under similarities; noisy inlier
    correspondences (0.3 px) on every overlapping pair; the start transforms
    are the true ones with corner errors of ~5-20 px (drift of chained pair
    transforms). The refinement brings every image within 1 px of the truth
    (the reference fixed) and the residual to the noise level."""
    rng = np.random.default_rng(4)
    world = []
    for r in range(2):
        for c in range(3):
            world.append(similarity(rng.uniform(-3, 3), rng.uniform(0.97, 1.03), 560.0 * c,
                                    420.0 * r))
    ref = 1
    G_true = [np.linalg.inv(world[ref]) @ world[k] for k in range(6)]
    corr = []
    for i in range(6):
        for j in range(i + 1, 6):
            Tij = np.linalg.inv(world[j]) @ world[i]
            p = np.c_[rng.uniform(0, 799, 3000), rng.uniform(0, 599, 3000)]
            q = (np.c_[p, np.ones(len(p))] @ Tij.T)
            q = q[:, :2] / q[:, 2:]
            inside = (q[:, 0] >= 0) & (q[:, 0] <= 799) & (q[:, 1] >= 0) & (q[:, 1] <= 599)
            if inside.sum() < 30:
                continue
            p, q = p[inside][:200], q[inside][:200]
            corr.append((i, j, p + rng.normal(0, 0.3, p.shape), q + rng.normal(0, 0.3, q.shape)))
    G0 = []
    for k in range(6):
        if k == ref:
            G0.append(np.eye(3))
            continue
        D = similarity(rng.uniform(-0.8, 0.8), rng.uniform(0.99, 1.01), rng.uniform(-8, 8),
                       rng.uniform(-8, 8))
        G0.append(D @ G_true[k])
    before = max(M.corner_error(G0[k], G_true[k], 800, 600) for k in range(6))
    G, info = M.refine(G0, corr, ref)
    after = max(M.corner_error(G[k], G_true[k], 800, 600) for k in range(6))
    assert before > 5.0
    assert after < 1.0, (before, after)
    assert np.array_equal(G[ref], np.eye(3))
    assert info["rms_after"] < 0.6 < info["rms_before"]


def test_refine_without_pairs_keeps_the_start():
    G0 = [np.eye(3), similarity(1, 1, 5, 5), None]
    G, info = M.refine(G0, [], 0)
    assert np.array_equal(G[1], G0[1]) and G[2] is None and info["iters"] == 0
