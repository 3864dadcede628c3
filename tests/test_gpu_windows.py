"""Window sets beyond the nested <= 128 px fast path, and matching by the
absolute threshold of Eq. 6 alone.

The paper's experiments (Table 2) use L sets such as {32, 40}, {32, 64},
{100, 128} and {256, 512} on images from 602x400 to 3072x4096; here they run
on seeded synthetic images of those sizes. Keypoints must equal the oracle's
bit for bit; orientations and descriptors follow the usual 1e-4 rules on a
sample; the Delta_s-only matcher follows match rule (i)."""
import numpy as np
import pytest

import oracle
import synth
import paper_2405_08578_amd as lp
from gpu_util import (angle_diff, assert_keypoints_equal, kp_numpy, match_margins,
                      oracle_features_at, orientation_ambiguity, rel_l2, say, to_dev)

pytestmark = pytest.mark.gpu


def texture(h, w, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = max(4, int(round(2000 * h * w / (2600 * 1600))))
    cv = synth.render_texture(0, 0, w, h, nb, rng)
    return synth.to_uint8(cv.tex, rng)


@pytest.mark.parametrize("h,w,Ls,seed", [
    (400, 602, [32, 40], 0),          # Table 2 sizes and window sets
    (490, 653, [32, 40], 1),
    (768, 1024, [32, 64], 2),          # nested: fast path
    (1080, 1920, [100, 128], 3),
    (3072, 4096, [256, 512], 4),
    (333, 517, [37], 5),               # one odd window size
    (300, 700, [64, 128, 256], 6),     # nested, largest above 128
    (77, 91, [5, 7, 9, 11, 13, 15, 17, 19], 7),
])
def test_detect_any_window_set(gpu, h, w, Ls, seed):
    img = texture(h, w, seed)
    say("detect window set", h, w, Ls)
    kps = lp.detect([to_dev(img, gpu)], lp.Params(Ls))
    assert_keypoints_equal(kp_numpy(kps[0]), oracle.detect(img, Ls))


def test_detect_batch_mixed_sizes_any_set(gpu):
    imgs = [texture(200, 300, 10), texture(97, 143, 11), texture(260, 180, 12)]
    Ls = [24, 40, 100]
    say("detect batch, window set", Ls)
    kps = lp.detect([to_dev(i, gpu) for i in imgs], lp.Params(Ls))
    for k, img in zip(kps, imgs):
        assert_keypoints_equal(kp_numpy(k), oracle.detect(img, Ls))


@pytest.mark.parametrize("h,w,Ls,seed,n_sample", [
    (490, 653, [32, 40], 1, 300),
    (1080, 1920, [100, 128], 3, 120),
    (3072, 4096, [256, 512], 4, 40),
])
def test_describe_any_window_set(gpu, h, w, Ls, seed, n_sample):
    img = texture(h, w, seed)
    say("describe window set", h, w, Ls)
    kps, th, de = lp.features([to_dev(img, gpu)], lp.Params(Ls))
    kpn = kp_numpy(kps[0])
    idx = np.sort(np.random.default_rng(seed).choice(len(kpn["x"]), min(n_sample, len(kpn["x"])),
                                                     replace=False))
    th_o, d_o, hist = oracle_features_at(img, kpn, Ls, idx)
    ok = orientation_ambiguity(hist) >= 1e-5
    assert ok.mean() >= 0.97
    g_th = th[0].cpu().numpy()[idx].astype(np.float64)
    g_de = de[0].cpu().numpy()[idx].astype(np.float64)
    assert np.all(angle_diff(g_th, th_o)[ok] < 1e-4)
    assert np.all(rel_l2(g_de, d_o)[ok] < 1e-4)


@pytest.mark.parametrize("prec", [0, 3])
def test_match_abs_threshold_only(gpu, prec):
    import torch
    rng = np.random.Generator(np.random.PCG64(31))
    B = synth.random_unit_rows(900, 128, rng).astype(np.float32)
    B[17] = B[5]                                   # duplicate: d1 == d2 for its copies
    A = synth.noisy_copies(B.astype(np.float64), rng.integers(0, 900, 700), 0.15,
                           rng).astype(np.float32)
    A[0] = B[5]
    tau = 0.45
    say("match, absolute threshold only", prec)
    r = lp.match([torch.from_numpy(A).to(gpu)], [torch.from_numpy(B).to(gpu)],
                 ratio=float("inf"), abs_thresh=tau, precision=prec)[0]
    g = {k: v.cpu().numpy() for k, v in r.items()}
    o = oracle.match(A.astype(np.float64), B.astype(np.float64), ratio=float("inf"),
                     abs_thresh=tau)
    # decided by d1 < tau alone: identical away from the threshold and from
    # nearest-neighbour ties (where only the index of equal distances differs)
    tie = match_margins(o["d1"], o["d2"], float("inf")) <= 1e-6
    safe = (np.abs(o["d1"] - tau) > 1e-5) & ~tie
    assert np.array_equal(g["match"][safe], o["match"][safe])
    assert g["match"][0] == 5                     # the duplicate is kept
    assert ((g["match"] >= 0) == (o["d1"] < tau))[np.abs(o["d1"] - tau) > 1e-5].all()
