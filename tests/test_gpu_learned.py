"""The learned-pruning path (score -> top 30 % -> describe the kept slots ->
match -> RANSAC) against the plain path on synthetic pairs with a known
homography, with the committed weights, and its fallback to the plain path.

Parity of each kernel is covered in test_gpu_scorer.py; here the criterion is
the method-level one: the learned path keeps nearly all of the plain path's
ground-truth-consistent matches. This is a quality check of the trained
weights, not parity (parity unpinned for the trained model)."""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from paper_2405_08578_amd import learned as L
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def load(gpu):
    w, _ = L.load_weights(L.DEFAULT_WEIGHTS, gpu)
    return w


def test_learned_keeps_matches_on_2600x1600_pair(gpu):
    pair = synth.config_pair(1)
    P = lp.Params([16, 32, 64, 128])
    imgs = [to_dev(pair.A, gpu), to_dev(pair.B, gpu)]
    say("learned vs plain, 2600x1600 pair")
    pl = L.run_pair(imgs, P, None, seed=1, H_true=pair.H)
    le = L.run_pair(imgs, P, load(gpu), seed=1, H_true=pair.H)
    assert le["path"] == "learned"
    assert le["gt_consistent"] >= 0.95 * pl["gt_consistent"]
    assert le["inliers"] >= 0.9 * pl["inliers"]
    assert pl["gt_consistent"] > 200
    # the learned path describes 30 % of the slots of each image
    res = L.learned_gpu(imgs, P, load(gpu))
    n = lp.num_keypoints(*pair.A.shape, P)
    assert [s.numel() for s in res["sel"]] == [lp.keep_count(n)] * 2


def test_fallback_when_pruning_fails(gpu):
    import torch
    pair = synth.config_pair(0)
    P = lp.Params([16, 32, 64])
    imgs = [to_dev(pair.A, gpu), to_dev(pair.B, gpu)]
    # constant scores: the prune degenerates to the first 30 % of slots (the
    # smallest windows of the top rows), and the inliers collapse
    zero = torch.zeros(20801, dtype=torch.float32, device=gpu)
    say("forced fallback")
    raw_res = L.learned_gpu(imgs, P, zero)
    k = lp.keep_count(lp.num_keypoints(*pair.A.shape, P))
    for s in raw_res["sel"]:
        assert np.array_equal(s.cpu().numpy(), np.arange(k))
    raw = L.finish(raw_res, seed=3)
    pl = L.run_pair(imgs, P, None, seed=3)
    assert raw["inliers"] < pl["inliers"]
    le = L.run_pair(imgs, P, zero, seed=3, min_inliers=raw["inliers"] + 1)
    assert le["path"] == "fallback"
    assert le["inliers"] == pl["inliers"] and le["matches"] == pl["matches"]


def test_batched_paths_equal_per_pair(gpu):
    pairs = [synth.config_pair(0), synth.make_mixed_pair((1100, 825, 430, 5))]
    P = lp.Params([16, 32, 64])
    imgs = [[to_dev(p.A, gpu), to_dev(p.B, gpu)] for p in pairs]
    w = load(gpu)
    say("batched plain / learned paths")
    bp = L.plain_gpu_batch(imgs, P)
    bl = L.learned_gpu_batch(imgs, P, w)
    for k, im in enumerate(imgs):
        sp = L.plain_gpu(im, P)
        sl = L.learned_gpu(im, P, w)
        assert np.array_equal(bp[k]["match"].cpu().numpy(), sp["match"].cpu().numpy())
        assert np.array_equal(bl[k]["match"].cpu().numpy(), sl["match"].cpu().numpy())
        for a, b in zip(bl[k]["sel"], sl["sel"]):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_batch_path_eager_and_graph_replays(gpu):
    # The preallocated step of both paths, run eagerly and as replays of one
    # captured graph (outputs clobbered and other eager work between the
    # replays), equals the allocating batch functions bit for bit.
    import torch
    pairs = [synth.config_pair(0), synth.make_mixed_pair((1100, 825, 430, 5))]
    P = lp.Params([16, 32, 64])
    imgs = [[to_dev(p.A, gpu), to_dev(p.B, gpu)] for p in pairs]
    w = load(gpu)
    say("batch path eager / graph")
    refs = {None: L.plain_gpu_batch(imgs, P), "w": L.learned_gpu_batch(imgs, P, w)}

    def same(res, ref):
        for a, b in zip(res, ref):
            assert np.array_equal(a["match"].cpu().numpy(), b["match"].cpu().numpy())
            for u, v in zip(a["kps"], b["kps"]):
                assert np.array_equal(u["x"].cpu().numpy(), v["x"].cpu().numpy())
            if "sel" in b:
                for u, v in zip(a["sel"], b["sel"]):
                    assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())

    for key, weights in ((None, None), ("w", w)):
        bp = L.BatchPath(imgs, P, weights=weights)
        bp.run()
        torch.cuda.synchronize()
        same(bp.results(), refs[key])
        bp.capture()
        for rep in range(3):
            for o in bp.out:
                o["match"].fill_(-7)
            if weights is not None:
                for s in bp.sel:
                    s.fill_(-7)
            L.plain_gpu_batch(imgs[:1], P)
            torch.cuda.synchronize()
            bp.replay()
            torch.cuda.synchronize()
            say("replay", key, rep)
            same(bp.results(), refs[key])
