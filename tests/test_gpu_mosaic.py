"""Mosaic registration of a shuffled tile set on the GPU path: all pairs
matched and their homographies found by the batched GPU RANSAC inside one
captured graph, then the rounds of Sec. 4 on the host. The synthetic tiles
carry their true world-to-tile homographies, so every registered tile's
placement is checked against the truth by the seam error (the distance, in
the reference frame, between where two overlapping tiles put the same
content): below 5 px on every link used for placement, and below 10 px on
every overlap once the transforms are refined jointly over all stitchable
pairs' inliers;
graph replays must reproduce the eager RANSAC results bit for bit."""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from paper_2405_08578_amd import mosaic as M
from paper_2405_08578_amd.allpairs import AllPairs
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def run_set(gpu, tiles, Ls, n_iter=2000):
    import torch
    imgs = [to_dev(t, gpu) for t in tiles.images]
    u = torch.from_numpy(synth.ransac_uniforms(n_iter, np.random.default_rng(5))).to(gpu)
    ap = AllPairs(imgs, lp.Params(Ls), ransac_uniforms=u)
    return ap


def check_registration(tiles, ap, min_inliers=12, link_px=5.0, overlap_px=10.0):
    H = ap.ransac["H"].cpu().numpy()
    st = ap.ransac["stats"].cpu().numpy()
    n = len(tiles.images)
    T, W = M.pair_transforms(n, ap.pairs, H, st[:, 1], st[:, 0], min_inliers=min_inliers)
    r = M.register(n, T, W)
    assert r["unregistered"] == []
    ref = r["reference"]
    G_true = [tiles.H_world[ref] @ np.linalg.inv(tiles.H_world[k]) for k in range(n)]
    seams = M.seam_errors(r["G"], G_true, [t.shape for t in tiles.images])
    # seams of the links that placed the images are aligned to a few pixels;
    # other overlaps accumulate the error of two placement chains (each pair
    # homography is fitted on its overlap strip only)
    for a, b in r["links"]:
        assert seams[(a, b)] < link_px, (a, b, seams[(a, b)])
    assert len(r["links"]) == n - 1
    # joint refinement over every stitchable pair's inliers: all overlaps,
    # not only the links, then agree to a few pixels (corner overlaps, which
    # no stitchable pair constrains directly, to overlap_px)
    kps = [{k: v.cpu().numpy() for k, v in kp.items()} for kp in ap.kps]
    corr = M.correspondences(ap.pairs, kps, [t.cpu().numpy() for t in ap.ransac["slotA"]],
                             [t.cpu().numpy() for t in ap.ransac["slotB"]],
                             [t.cpu().numpy() for t in ap.ransac["inlier"]], st, W)
    G, info = M.refine(r["G"], corr, ref)
    seams_r = M.seam_errors(G, G_true, [t.shape for t in tiles.images])
    assert max(seams_r.values()) < overlap_px, seams_r
    assert max(seams_r.values()) < max(seams.values())
    assert info["rms_after"] <= info["rms_before"]
    print("seams chained", max(seams.values()), "refined", max(seams_r.values()), info,
          flush=True)
    return r, seams


def test_small_tiles_graph_registration(gpu):
    import torch
    tiles = synth.make_tiles(world_w=2000, world_h=1300, tile_w=(760, 800), tile_h=(480, 520),
                             seed=8)
    ap = run_set(gpu, tiles, [16, 32, 64], n_iter=16384)
    say("mosaic small tiles, eager")
    ap.run()
    torch.cuda.synchronize()
    H0 = ap.ransac["H"].cpu().numpy().copy()
    s0 = ap.ransac["stats"].cpu().numpy().copy()
    check_registration(tiles, ap, min_inliers=18, link_px=10.0)   # ~30 inliers per link
    say("mosaic small tiles, graph")
    ap.capture()
    for _ in range(2):
        ap.ransac["H"].fill_(7.0)
        ap.ransac["stats"].fill_(-9)
        torch.cuda.synchronize()
        ap.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ap.ransac["H"].cpu().numpy(), H0)
        assert np.array_equal(ap.ransac["stats"].cpu().numpy(), s0)


def test_full_tiles_registration(gpu):
    import torch
    tiles = synth.make_tiles()
    ap = run_set(gpu, tiles, [16, 32, 64, 128], n_iter=16384)
    say("mosaic full tiles")
    ap.capture()
    ap.replay()
    torch.cuda.synchronize()
    r, seams = check_registration(tiles, ap)
    print("rounds", r["rounds"], "seam errors", seams)
