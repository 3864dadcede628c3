"""Batched GPU RANSAC (lpsift_ransac) against the FP64 oracle (oracle/ransac.py)
on the same compacted matches and the same uniform draws.

Rules: the compacted slot lists are exact; the chosen hypothesis is the
oracle's (hypothesis solves differ only by rounding: closed-form basis
solution on the GPU, least squares in the oracle, so inlier counts can differ
only through points within rounding of the threshold, and tests use data
where none is); the refitted H maps the image corners within 1e-6 px of the
oracle's; the inlier masks are equal for every match whose oracle error is
more than 1e-6 px from the threshold."""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from oracle import ransac as R
from gpu_util import kp_numpy, say, to_dev

pytestmark = pytest.mark.gpu

THRESH = 3.0


def oracle_for(kA, kB, m, u, selA=None, selB=None):
    qi = np.nonzero(m >= 0)[0]
    sa = qi if selA is None else selA[qi]
    sb = m[qi] if selB is None else selB[m[qi]]
    pa = np.stack([kA["x"][sa], kA["y"][sa]], 1).astype(np.float64)
    pb = np.stack([kB["x"][sb], kB["y"][sb]], 1).astype(np.float64)
    S = R.samples_from_uniforms(u, len(pa))
    H, mask, best = R.ransac(pa, pb, S, THRESH)
    return sa, sb, pa, pb, H, mask, best


def check(g, p, kA, kB, m, u, selA=None, selB=None, corners=(640, 480)):
    sa, sb, pa, pb, H, mask, best = oracle_for(kA, kB, m, u, selA, selB)
    st = g["stats"][p].cpu().numpy()
    n = len(sa)
    assert st[0] == n
    assert np.array_equal(g["slotA"][p].cpu().numpy()[:n], sa)
    assert np.array_equal(g["slotB"][p].cpu().numpy()[:n], sb)
    assert st[2] == best
    if best < 0:
        assert st[1] == 0 and np.all(g["H"][p].cpu().numpy() == 0)
        return
    Hg = g["H"][p].cpu().numpy().reshape(3, 3)
    w, h = corners
    c = np.array([[0, 0], [w - 1, 0], [w - 1, h - 1], [0, h - 1]], np.float64)
    qg, wg = R.apply(Hg, c)
    qo, wo = R.apply(H, c)
    assert np.max(np.abs(qg / wg[:, None] - qo / wo[:, None])) < 1e-6
    err = R.reprojection_error(H, pa, pb)
    far = np.abs(err - THRESH) > 1e-6
    gm = g["inlier"][p].cpu().numpy()[:n].astype(bool)
    assert np.array_equal(gm[far], mask[far])
    assert st[1] == gm.sum()


def planted(n_in, n_out, seed, w=640, h=480):
    rng = np.random.default_rng(seed)
    Ht = np.array([[1.05, 0.08, 40.0], [-0.06, 0.97, -25.0], [2e-5, -1e-5, 1.0]])
    xa = rng.integers(0, w, n_in + n_out)
    ya = rng.integers(0, h, n_in + n_out)
    q = np.c_[xa, ya, np.ones(len(xa))] @ Ht.T
    xb = np.rint(q[:, 0] / q[:, 2]).astype(np.int64)
    yb = np.rint(q[:, 1] / q[:, 2]).astype(np.int64)
    out = rng.permutation(n_in + n_out)[:n_out]
    xb[out] = rng.integers(0, w, n_out)
    yb[out] = rng.integers(0, h, n_out)
    return xa, ya, xb, yb


def kp_tensors(x, y, gpu):
    import torch
    n = len(x)
    k = lp.empty_keypoints(n, gpu)
    k["x"].copy_(torch.from_numpy(np.asarray(x, np.int32)))
    k["y"].copy_(torch.from_numpy(np.asarray(y, np.int32)))
    return k


@pytest.mark.parametrize("n_in,n_out,seed", [(300, 700, 0), (50, 20, 1), (4, 0, 2), (3, 5, 3),
                                             (0, 0, 4), (900, 100, 5)])
def test_planted_correspondences(gpu, n_in, n_out, seed):
    import torch
    xa, ya, xb, yb = planted(n_in, n_out, seed)
    n = len(xa)
    rng = np.random.default_rng(10 + seed)
    # query i matches registered row perm[i]; every 5th query rejected
    perm = rng.permutation(n)
    kA = kp_tensors(xa, ya, gpu)
    kB = kp_tensors(xb[np.argsort(perm)], yb[np.argsort(perm)], gpu)
    m = perm.astype(np.int32)
    m[::5] = -1
    u = synth.ransac_uniforms(1000, np.random.default_rng(seed))
    say("gpu ransac planted", n_in, n_out)
    g = lp.ransac_gpu([kA], [kB], [torch.from_numpy(m).to(gpu)],
                      torch.from_numpy(u).to(gpu), THRESH)
    check(g, 0, kp_numpy(kA), kp_numpy(kB), m, u)


def test_real_pair_and_selected_slots(gpu):
    import torch
    from paper_2405_08578_amd import learned as L
    pair = synth.config_pair(0)
    P = lp.Params([16, 32, 64])
    imgs = [to_dev(pair.A, gpu), to_dev(pair.B, gpu)]
    u = synth.ransac_uniforms(2000, np.random.default_rng(7))
    tu = torch.from_numpy(u).to(gpu)
    say("gpu ransac, plain and learned lists")
    pl = L.plain_gpu(imgs, P)
    w, _ = L.load_weights(L.DEFAULT_WEIGHTS, gpu)
    le = L.learned_gpu(imgs, P, w)
    kA = [pl["kps"][0], le["kps"][0]]
    kB = [pl["kps"][1], le["kps"][1]]
    g = lp.ransac_gpu(kA, kB, [pl["match"], le["match"]], tu, THRESH,
                      selA=[torch.arange(pl["kps"][0]["x"].numel(), dtype=torch.int32, device=gpu),
                            le["sel"][0]],
                      selB=[torch.arange(pl["kps"][1]["x"].numel(), dtype=torch.int32, device=gpu),
                            le["sel"][1]])
    check(g, 0, kp_numpy(pl["kps"][0]), kp_numpy(pl["kps"][1]), pl["match"].cpu().numpy(), u)
    check(g, 1, kp_numpy(le["kps"][0]), kp_numpy(le["kps"][1]), le["match"].cpu().numpy(), u,
          le["sel"][0].cpu().numpy(), le["sel"][1].cpu().numpy())
    st = g["stats"].cpu().numpy()
    assert st[0, 1] > 30 and st[1, 1] > 30
    # the recovered homography is the generator's
    Hg = g["H"][0].cpu().numpy().reshape(3, 3)
    c = np.array([[100.0, 100.0], [500.0, 100.0], [300.0, 400.0]])
    ptg = np.c_[c, np.ones(3)] @ Hg.T
    ptt = np.c_[c, np.ones(3)] @ pair.H.T
    assert np.max(np.abs(ptg[:, :2] / ptg[:, 2:] - ptt[:, :2] / ptt[:, 2:])) < 2.0


def test_batch_of_many_pairs_equals_single(gpu):
    import torch
    u = synth.ransac_uniforms(700, np.random.default_rng(3))
    tu = torch.from_numpy(u).to(gpu)
    kA, kB, ms = [], [], []
    for s in range(19):                                 # two launches
        xa, ya, xb, yb = planted(80 + 7 * s, 40 + 3 * s, 100 + s)
        kA.append(kp_tensors(xa, ya, gpu))
        kB.append(kp_tensors(xb, yb, gpu))
        m = np.arange(len(xa), dtype=np.int32)
        m[s % 4::7] = -1
        ms.append(torch.from_numpy(m).to(gpu))
    say("gpu ransac, 19 pairs")
    g = lp.ransac_gpu(kA, kB, ms, tu, THRESH)
    for p in range(19):
        one = lp.ransac_gpu([kA[p]], [kB[p]], [ms[p]], tu, THRESH)
        assert np.array_equal(one["H"].cpu().numpy()[0], g["H"].cpu().numpy()[p])
        assert np.array_equal(one["stats"].cpu().numpy()[0], g["stats"].cpu().numpy()[p])
        check(g, p, kp_numpy(kA[p]), kp_numpy(kB[p]), ms[p].cpu().numpy(), u)
