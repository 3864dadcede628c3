"""GPU parity of lpsift_detect against the FP64 oracle: bit-exact keypoints."""
import numpy as np
import pytest

import oracle
import synth
import paper_2405_08578_amd as lp
from gpu_util import assert_keypoints_equal, kp_numpy, say, to_dev

pytestmark = pytest.mark.gpu


CASES = [
    # (h, w, Ls, levels, seed): ragged sizes, tiny images, heavy ties
    (1, 1, [4], 256, 0),
    (5, 7, [4, 8], 3, 1),
    (17, 33, [4, 8, 16], 256, 2),
    (100, 129, [16, 32, 64, 128], 2, 3),
    (257, 300, [16, 32, 64, 128], 256, 4),
    (130, 260, [16, 48], 256, 5),
    (64, 64, [8, 24, 48], 4, 6),
    (480, 640, [16, 32, 64], 1, 7),            # constant image
    (300, 515, [4, 8, 16, 32, 64, 128], 256, 8),
    (250, 333, [12, 24], 256, 9),             # 120-px tiles, 8-bit packed row/column codes
    (161, 320, [20, 40, 120], 3, 10),         # first side 20: 5-bit columns
]


@pytest.mark.parametrize("h,w,Ls,levels,seed", CASES)
def test_detect_random_images(gpu, h, w, Ls, levels, seed):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, levels, (h, w)).astype(np.uint8)
    say("detect", h, w, Ls, levels, seed)
    kp = lp.detect([to_dev(img, gpu)], lp.Params(Ls))[0]
    assert_keypoints_equal(kp_numpy(kp), oracle.detect(img, Ls))


def test_detect_pitched_and_unaligned_views(gpu):
    import torch
    rng = np.random.default_rng(11)
    big = rng.integers(0, 256, (200, 301)).astype(np.uint8)
    t = to_dev(big, gpu)
    view = t[3:190, 5:290]                     # pitch 301, data not 4-byte aligned
    say("detect view", tuple(view.shape), view.stride())
    kp = lp.detect([view], lp.Params([16, 32, 64]))[0]
    assert_keypoints_equal(kp_numpy(kp), oracle.detect(big[3:190, 5:290], [16, 32, 64]))


def test_detect_batch_equals_single(gpu):
    rng = np.random.default_rng(12)
    imgs = [rng.integers(0, 256, (h, w)).astype(np.uint8)
            for h, w in [(480, 640), (77, 1000), (1024, 33), (128, 128)] * 5]  # 20 > one launch
    P = lp.Params([16, 32, 64, 128])
    say("detect batch", len(imgs))
    kps = lp.detect([to_dev(i, gpu) for i in imgs], P)
    for img, kp in zip(imgs, kps):
        assert_keypoints_equal(kp_numpy(kp), oracle.detect(img, P.L))


@pytest.mark.parametrize("cfg", [0, 1])
def test_detect_config_pairs(gpu, cfg):
    pair = synth.config_pair(cfg)
    Ls = [16, 32, 64] if cfg == 0 else [16, 32, 64, 128]
    say("detect config pair", cfg)
    kps = lp.detect([to_dev(pair.A, gpu), to_dev(pair.B, gpu)], lp.Params(Ls))
    for img, kp in zip((pair.A, pair.B), kps):
        g = kp_numpy(kp)
        assert len(g["x"]) == (3160 if cfg == 0 else 43396)
        assert_keypoints_equal(g, oracle.detect(img, Ls))


def test_detect_deterministic(gpu):
    pair = synth.config_pair(0)
    t = to_dev(pair.A, gpu)
    P = lp.Params([16, 32, 64])
    a = kp_numpy(lp.detect([t], P)[0])
    b = kp_numpy(lp.detect([t], P)[0])
    for f in a:
        assert np.array_equal(a[f], b[f])
