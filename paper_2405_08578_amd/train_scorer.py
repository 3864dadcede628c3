"""Train the learned keypoint scorer on seeded synthetic pairs.

    python -m paper_2405_08578_amd.train_scorer --pairs 500 --steps 24000 \
        --out paper_2405_08578_amd/scorer/lpsift_scorer_v2

Pairs are generated like the 2600x1600 benchmark pair (instances 100 ..
100 + pairs - 1 of that configuration, disjoint from the benchmark's instance
0) by a pool of host processes. Each pair runs the plain GPU path and host
RANSAC; the inlier endpoints are the positives (see learned.pair_records).
Training runs lpsift_scorer_train_step with class-balanced weights. A few
held-out pairs (instances 900 ..) then compare the learned path's RANSAC
inliers with the plain path's (the share of the plain inliers, as slot pairs,
that the learned path keeps); the result goes into the weight file's
metadata.
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time


def _make(instance):
    import synth
    p = synth.config_pair(1, instance)
    return instance, p.A, p.B, p.H


def log(*a):
    print("[train]", *a, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=500)
    ap.add_argument("--steps", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=0.05,
                    help="final step size as a fraction of --lr (half-cosine decay)")
    ap.add_argument("--neg-per-pos", type=int, default=4)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--eval-pairs", type=int, default=16)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    ctx = mp.get_context("spawn")
    pool = ctx.Pool(args.workers)          # host processes only: no GPU in the workers

    import numpy as np
    import torch
    import synth
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd import learned as L

    dev = torch.device("cuda:0")
    P = lp.Params([16, 32, 64, 128])
    t0 = time.time()
    pats, exts, labs = [], [], []
    inl = []
    insts = list(range(100, 100 + args.pairs))
    for k, (inst, A, B, _) in enumerate(pool.imap(_make, insts, chunksize=1)):
        imgs = [torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)]
        pa, ex, la, n_in = L.pair_records(imgs, P, seed=inst, neg_per_pos=args.neg_per_pos)
        pats.append(pa)
        exts.append(ex)
        labs.append(la)
        inl.append(n_in)
        if k % 25 == 0 or k == len(insts) - 1:
            log(f"pair {k + 1}/{len(insts)} inliers {n_in} records {sum(int(x.numel()) for x in labs)}"
                f" ({time.time() - t0:.0f} s)")
    patches = torch.cat(pats)
    extra = torch.cat(exts)
    labels = torch.cat(labs)
    del pats, exts, labs
    n_pos = int(labels.sum().item())
    log(f"records {labels.numel()} positives {n_pos}")

    init = synth.scorer_init(np.random.default_rng(args.seed))
    w, losses = L.train(patches, extra, labels, init, args.steps, args.batch, args.lr,
                        seed=args.seed, log=log, lr_final=args.lr_final)
    torch.cuda.synchronize()

    # held-out comparison: learned (no fallback) vs plain; retention = the
    # plain path's RANSAC inliers (slot pairs) that the learned path keeps
    ev = []
    evi = list(range(900, 900 + args.eval_pairs))
    for inst, A, B, H in pool.imap(_make, evi, chunksize=1):
        imgs = [torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)]
        pl = L.run_pair(imgs, P, None, seed=inst, H_true=H)
        le = L.run_pair(imgs, P, w, seed=inst, min_inliers=0, H_true=H)
        kept, tot = L.inlier_retention(pl, le)
        ev.append((inst, pl["inliers"], le["inliers"], pl["gt_consistent"], le["gt_consistent"],
                   kept))
        log(f"held-out {inst}: RANSAC inliers plain {pl['inliers']} learned {le['inliers']} "
            f"kept {kept}; ground-truth-consistent matches plain {pl['gt_consistent']} learned "
            f"{le['gt_consistent']}")
    pool.close()
    pool.join()
    tot_p = sum(e[1] for e in ev)
    tot_l = sum(e[2] for e in ev)
    gt_p = sum(e[3] for e in ev)
    gt_l = sum(e[4] for e in ev)
    kept_all = sum(e[5] for e in ev)
    meta = {"train_pairs": args.pairs, "train_instances": [insts[0], insts[-1]],
            "pair_config": "2600x1600 blob-texture pairs, random similarity, IoU 0.3-0.5",
            "L": [16, 32, 64, 128], "records": int(labels.numel()), "positives": n_pos,
            "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "lr_final": args.lr_final, "neg_per_pos": args.neg_per_pos, "seed": args.seed,
            "loss_history": losses,
            "ransac_iters": L.RANSAC_ITERS, "ransac_refine_rounds": L.REFINE_ROUNDS,
            "heldout": [dict(zip(("instance", "ransac_plain", "ransac_learned", "gt_plain",
                                  "gt_learned", "plain_inliers_kept"), e)) for e in ev],
            "heldout_inlier_retention": (kept_all / tot_p) if tot_p else None,
            "heldout_inlier_retention_min_pair": min(e[5] / max(e[1], 1) for e in ev) if ev else None,
            "heldout_inlier_count_ratio": (tot_l / tot_p) if tot_p else None,
            "heldout_gt_match_retention": (gt_l / gt_p) if gt_p else None}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    L.save_weights(args.out, w.cpu().numpy(), meta)
    log(f"saved {args.out}.bin / .json; held-out retention of the plain RANSAC inliers "
        f"{meta['heldout_inlier_retention']} (lowest pair "
        f"{meta['heldout_inlier_retention_min_pair']}), inlier count ratio "
        f"{meta['heldout_inlier_count_ratio']}, ground-truth-consistent matches "
        f"{meta['heldout_gt_match_retention']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
