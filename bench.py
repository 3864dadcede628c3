#!/usr/bin/env python3
"""Throughput of the LP-SIFT hot path on one MI355X.

One step = detect + orient + describe both images of a 2600x1600 uint8 pair
(L = 16, 32, 64, 128) and match every reference descriptor against the
registered set with the 0.8 ratio test: the whole GPU hot path for one pair,
inputs resident in HBM before the timed region.

Prints ONE JSON line: value = pairs/s; detect+describe Mpix/s as a side field;
per-kernel device times from the library's timing facility (HIP events
recorded around every launch on the stream it runs on) and from them a roofline
object for the dominant kernel (the FP32 matrix-core contraction of the
matcher); side fields for the reduced-precision matchers and for the 9-tile
all-pairs workload (tuned work split, HIP-graph replay) and for learned
keypoint pruning against the plain path on 32 mixed-size pairs; and the FP64
oracle timed on a bounded sample on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-tiles]
                    [--no-learned]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s detect+describe; pairs/s matched; learned-pruned vs plain, equal inliers"
PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0           # GB/s
PEAK_INT8_MFMA = 5000.0     # TOP/s, MI355X dense int8 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tiles", action="store_true",
                    help="skip the 9-tile all-pairs side measurement")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-pruning side measurement (32 mixed-size pairs)")
    ap.add_argument("--learned-pairs", type=int, default=32)
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="runs of the oracle on the whole pair for the CPU baseline")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before warm-up, copy a buffer of this size once (untimed): a plain "
                         "copy kernel of known traffic for calibrating HBM counters")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_topk_f32_2600x1600_pair_traffic.md")
MATCH_SRC = os.path.join(ROOT, "paper_2405_08578_amd", "csrc", "match.hip")
DESC_COUNTERS_FILE = os.path.join(ROOT, "profiles", "orient_describe_2600x1600_pair_counters.md")
DESC_SRC = os.path.join(ROOT, "paper_2405_08578_amd", "csrc", "describe.hip")
# VALU issue ceiling: 1,024 SIMDs x 2.4 GHz, one wave64 VALU instruction per
# 4 cycles on a 16-lane SIMD
PEAK_VALU_GINSTR = 1024 * 2.4 / 4


def committed_figure(path, src, src_key, key):
    """A figure from a committed PMC summary ("- key: value" lines), or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get(src_key) != sha:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch of the contraction kernel from the committed PMC
    summary, or None when the kernel source changed since it was taken."""
    return committed_figure(TRAFFIC_FILE, MATCH_SRC, "match.hip sha256", "traffic bytes per launch")


def describe_valu_instructions():
    """Wave-level VALU instructions of the describe step on the pair (both
    images), from the committed counter summary; None when stale."""
    return committed_figure(DESC_COUNTERS_FILE, DESC_SRC, "describe.hip sha256",
                            "VALU instructions per pair step")


def cpu_baseline(pair, Ls, reps=3):
    """The FP64 oracle on the host, the whole pair: detect+orient+describe
    both images and the brute-force matcher over every reference descriptor;
    `reps` runs, the median time per pair."""
    import numpy as np
    import oracle
    times, t_dd, t_m = [], [], []
    nA = nB = 0
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, dA = oracle.features(pair.A, Ls)
        _, _, dB = oracle.features(pair.B, Ls)
        t1 = time.perf_counter()
        oracle.match(dA, dB)
        t2 = time.perf_counter()
        t_dd.append(t1 - t0)
        t_m.append(t2 - t1)
        times.append(t2 - t0)
        nA, nB = len(dA), len(dB)
    t_pair = float(np.median(times))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / t_pair, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle, the whole {pair.A.shape[1]}x{pair.A.shape[0]} pair {reps} "
                       f"times: detect+describe of both images (median {np.median(t_dd):.2f} s) "
                       f"+ brute-force match of all {nA} reference descriptors vs {nB} "
                       f"(median {np.median(t_m):.2f} s)"),
            "seconds_per_pair": t_pair}


def kernel_table(t, steps):
    """Mean device ms per step and per launch of each timed kernel."""
    return {k: {"ms_per_step": round(v["ms"] / steps, 4),
                "launches_per_step": v["launches"] / steps,
                "ms_per_launch": round(v["ms"] / max(v["launches"], 1), 4)}
            for k, v in t.items() if v["launches"] > 0}


def timed(fn, steps, stream):
    """Wall-clock and event ms per call of fn over `steps` calls."""
    import torch
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e[0].record(stream)
    for _ in range(steps):
        fn()
    e[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return 1000.0 * wall / steps, e[0].elapsed_time(e[1]) / steps


def bench_tiles(args, dev):
    """All-pairs matching of the 9 shuffled tiles: detect + describe all tiles
    and match all 36 pairs (i < j) per step, the work split tuned on the
    device, the step captured in a HIP graph and replayed."""
    import numpy as np
    import torch
    import synth
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd.allpairs import AllPairs

    tiles = synth.make_tiles()
    Ls = [16, 32, 64, 128]
    P = lp.Params(Ls)
    imgs = [torch.from_numpy(t).to(dev) for t in tiles.images]
    stream = torch.cuda.current_stream()
    steps = max(2, args.steps // 2)
    res = {"workload": "9 shuffled uint8 tiles 2600-2800 x 1600-1800 cut from a 7000x4500 "
                       "synthetic world (3x3 grid, 25-35 % overlaps, per-tile similarity and "
                       "gain): detect+orient+describe all tiles, FP32 match of all 36 pairs "
                       "(i < j) with ratio 0.8",
           "tile_shapes": [list(t.shape) for t in tiles.images], "pairs": 36, "L": Ls}

    # tune the candidate-range split on the real descriptor sets
    ap = AllPairs(imgs, P, precision=0)
    ap.run()
    torch.cuda.synchronize()
    A = [ap.desc[i] for i, _ in ap.pairs]
    B = [ap.desc[j] for _, j in ap.pairs]
    tunes = {}
    for prec in (0, 3):
        tunes[prec] = lp.match_tune(A, B, precision=prec, candidates=(1, 2, 3, 4, 6, 8), reps=1)
    res["tuned_b_chunks"] = {"fp32": tunes[0]["b_chunks"], "split": tunes[3]["b_chunks"]}
    res["tune_ms"] = {"fp32": [round(v, 2) for v in tunes[0]["ms"]],
                      "split": [round(v, 2) for v in tunes[3]["ms"]],
                      "candidates": tunes[0]["candidates"]}
    del A, B, ap
    torch.cuda.empty_cache()

    n_kp = [lp.num_keypoints(t.shape[0], t.shape[1], P) for t in imgs]
    flops = sum(2.0 * n_kp[i] * n_kp[j] * 128 for i, j in
                [(i, j) for i in range(9) for j in range(i + 1, 9)])
    ref_lists = None
    variants = {}
    for prec, name in ((0, "fp32"), (3, "split_bf16x3_certified"), (1, "bf16"), (2, "fp8")):
        bc = tunes[prec]["b_chunks"] if prec in tunes else 0
        ap = AllPairs(imgs, P, precision=prec, b_chunks=bc)
        for _ in range(max(1, args.warmup)):
            ap.run()
        eager_wall, eager_ev = timed(ap.run, steps, stream)
        # per-kernel device time of one eager step
        lp.timing_enable(True)
        ap.run()
        kt = kernel_table(lp.timing_read(), 1)
        lp.timing_enable(False)
        ap.capture()
        for _ in range(max(1, args.warmup)):
            ap.replay()
        wall, ev = timed(ap.replay, steps, stream)
        lists = [o["match"].cpu().numpy() for o in ap.out]
        v = {"ms_per_step_graph": round(wall, 3), "ms_per_step_eager": round(eager_wall, 3),
             "pairs_per_s": round(36 * 1000.0 / wall, 3),
             "detect_describe_match_mpix_per_s": round(ap.megapixels * 1000.0 / wall, 1),
             "kernels": kt}
        key = {0: "match_fp32", 3: "match_split"}.get(prec, "match_lowp")
        if key in kt:
            v["contraction_tflops" + ("" if prec == 0 else "_equiv")] = round(
                flops / (kt[key]["ms_per_step"] * 1e-3) / 1e12, 1)
        if prec == 3:
            v["queries_rematched_fp32"] = int(ap.stats.item())
        if ref_lists is None:
            ref_lists = lists
            v["matches"] = int(sum((m >= 0).sum() for m in lists))
        else:
            same = sum(int((a == b).sum()) for a, b in zip(lists, ref_lists))
            v["list_agreement_with_fp32"] = round(same / sum(len(m) for m in lists), 6)
        variants[name] = v
        del ap
        torch.cuda.empty_cache()
    # exact uint8 variant of the step (quantise all 9 sets, integer match of
    # every pair), graph-replayed
    ap = AllPairs(imgs, P, u8=True)
    ap.capture()
    for _ in range(max(1, args.warmup)):
        ap.replay()
    wall, _ = timed(ap.replay, steps, stream)
    lp.timing_enable(True)
    ap.run()
    kt = kernel_table(lp.timing_read(), 1)
    lp.timing_enable(False)
    same = sum(int((o["match"].cpu().numpy() == r).sum()) for o, r in zip(ap.out, ref_lists))
    ops = sum(2.0 * n_kp[i] * n_kp[j] * 128 for i, j in ap.pairs)
    k_ms = kt["match_u8"]["ms_per_step"]
    variants["uint8_exact"] = {
        "ms_per_step_graph": round(wall, 3), "pairs_per_s": round(36 * 1000.0 / wall, 3),
        "kernels": kt, "contraction_int8_tops": round(ops / (k_ms * 1e-3) / 1e12, 1),
        "matches": int(sum(int((o["match"] >= 0).sum().item()) for o in ap.out)),
        "list_agreement_with_fp32": round(same / sum(len(m) for m in ref_lists), 6)}
    del ap
    torch.cuda.empty_cache()
    res["descriptors"] = int(sum(n_kp))
    res["match_gflop_per_step"] = round(flops / 1e9, 1)
    res["variants"] = variants

    # mosaic registration: the FP32 all-pairs step plus the batched GPU RANSAC
    # of all 36 pairs in one graph, then the rounds of Sec. 4 on the host
    from paper_2405_08578_amd import mosaic as M
    n_iter = 16384
    u = torch.from_numpy(synth.ransac_uniforms(n_iter, np.random.default_rng(11))).to(dev)
    ap = AllPairs(imgs, P, precision=0, b_chunks=tunes[0]["b_chunks"], ransac_uniforms=u)
    ap.capture()
    for _ in range(max(1, args.warmup)):
        ap.replay()
    wall, _ = timed(ap.replay, steps, stream)
    lp.timing_enable(True)
    ap.run()
    kt = kernel_table(lp.timing_read(), 1)
    lp.timing_enable(False)
    t0 = time.perf_counter()
    H = ap.ransac["H"].cpu().numpy()
    st = ap.ransac["stats"].cpu().numpy()
    T, W = M.pair_transforms(len(imgs), ap.pairs, H, st[:, 1], st[:, 0])
    reg = M.register(len(imgs), T, W)
    host_ms = 1000.0 * (time.perf_counter() - t0)
    ref = reg["reference"]
    G_true = [tiles.H_world[ref] @ np.linalg.inv(tiles.H_world[k]) for k in range(len(imgs))]
    seams = M.seam_errors(reg["G"], G_true, [t.shape for t in tiles.images])
    link = [seams[(a, b)] for a, b in reg["links"]]
    res["registration"] = {
        "what": "9 tiles: detect+describe, FP32 match of 36 pairs, GPU RANSAC (16384 "
                "hypotheses per pair, 3 px) in one graph replay; then H_M rounds on the host",
        "ms_per_step_graph": round(wall, 3), "host_rounds_ms": round(host_ms, 3),
        "ransac_ms": kt.get("ransac", {}).get("ms_per_step"),
        "registered": len(imgs) - len(reg["unregistered"]),
        "stitchable_pairs": int((W > 0).sum() // 2),
        "inliers_on_links": [int(W[a, b]) for a, b in reg["links"]],
        "max_link_seam_px": round(max(link), 3) if link else None,
        "max_overlap_seam_px": round(max(seams.values()), 3) if seams else None,
        "paper_context": "the paper stitches nine images over 2600x1600 in 158.94 s "
                         "(MATLAB on an Intel i9-12900, including warping and blending; "
                         "here they are the warp_blend figures)"}

    # warp and blend the registered tiles into the reference frame's canvas
    idx = [k for k in range(len(imgs)) if reg["G"][k] is not None]
    Gs = [reg["G"][k] for k in idx]
    wimgs = [imgs[k] for k in idx]
    x0, y0, cw, ch = M.canvas_bounds([tuple(t.shape) for t in wimgs], Gs)
    canvas = torch.empty((ch, cw), dtype=torch.float32, device=dev)
    count = torch.empty((ch, cw), dtype=torch.uint8, device=dev)
    wcall = lambda: lp.warp_blend(wimgs, Gs, x0, y0, cw, ch, canvas=canvas, count=count,
                                  stream=stream)
    for _ in range(max(1, args.warmup)):
        wcall()
    _, wms = timed(wcall, args.steps, stream)
    lp.timing_enable(True)
    timed(wcall, args.steps, stream)
    kw = kernel_table(lp.timing_read(), args.steps)
    lp.timing_enable(False)
    est, est_count = canvas.clone(), count.clone()
    lp.warp_blend(wimgs, [G_true[k] for k in idx], x0, y0, cw, ch, canvas=canvas, count=count,
                  stream=stream)
    both = (count > 0) & (est_count > 0)
    diff = (est - canvas).abs()[both]
    wbytes = cw * ch * 5 + sum(int(t.numel()) for t in wimgs)
    res["registration"]["warp_blend"] = {
        "canvas": [cw, ch], "images": len(wimgs),
        "ms": round(wms, 4), "kernel_ms": kw["warp"]["ms_per_launch"],
        "algorithmic_GBps": round(wbytes / (kw["warp"]["ms_per_launch"] * 1e-3) / 1e9, 1),
        "covered_share": round(both.float().mean().item(), 4),
        "mean_abs_diff_vs_true_transforms": round(diff.mean().item(), 3),
        "end_to_end_ms": round(wall + host_ms + wms, 3)}
    del canvas, count, est, est_count
    del ap
    torch.cuda.empty_cache()
    return res


def bench_learned(args, dev, pairs):
    """Learned pruning vs the plain path on mixed-size pairs (1024x768 ..
    4000x3000): GPU pairs/s of both paths over all pairs at once (every image
    in the same detect/score/prune/describe calls, all pairs in one match
    call; inputs resident), then host RANSAC on both results; the learned path
    falls back to the plain path for a pair whose RANSAC keeps fewer than 12
    inliers."""
    import numpy as np
    import torch
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd import learned as L

    w, info = L.load_weights(L.DEFAULT_WEIGHTS, dev)
    P = lp.Params([16, 32, 64, 128])
    imgs = [[torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev)] for p in pairs]
    mpix = sum(2 * p.A.size for p in pairs) / 1e6

    # Both paths with every buffer allocated once (BatchPath), timed eagerly
    # (the binding marshals 64 images per call on the host) and as replays of
    # one captured HIP graph (the GPU work alone); the graph figures are the
    # reported pairs/s of both paths.
    steps = max(1, min(3, args.steps // 5))

    def timed(bp):
        bp.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bp.run()
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1000.0 / steps
        bp.capture()
        bp.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bp.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / steps, eager_ms

    out = {}
    lists = {}
    for name, weights in (("plain", None), ("learned", w)):
        bp = L.BatchPath(imgs, P, weights=weights)
        g_ms, e_ms = timed(bp)
        out[name] = (g_ms, bp.results(), e_ms)
        lists[name] = [o["match"].cpu().numpy() for o in bp.out]
        del bp
    # the same two paths with the certified split-BF16 matcher (its lists
    # equal the FP32 path's): graph replays only, lists compared
    split = {}
    for name, weights in (("plain", None), ("learned", w)):
        bp = L.BatchPath(imgs, P, weights=weights, precision=3)
        g_ms, _ = timed(bp)
        same = sum(int((o["match"].cpu().numpy() == m).sum()) for o, m in zip(bp.out, lists[name]))
        total = sum(len(m) for m in lists[name])
        split[name] = (g_ms, same / max(total, 1))
        del bp
    torch.cuda.empty_cache()
    rows = []
    t0 = time.perf_counter()
    for k, p in enumerate(pairs):
        pl = L.finish(out["plain"][1][k], seed=k, H_true=p.H)
        le = L.finish(out["learned"][1][k], seed=k, H_true=p.H)
        fb = le["inliers"] < 12
        if fb:
            le = pl
        rows.append((pl["inliers"], le["inliers"], pl["gt_consistent"], le["gt_consistent"], fb,
                     pl["matches"], le["matches"]))
    t_host = (time.perf_counter() - t0) / (2 * len(pairs))
    r = np.array(rows, dtype=np.float64)
    ms_p, ms_l = out["plain"][0], out["learned"][0]
    return {"workload": f"{len(pairs)} mixed-size pairs (widths 1024-4000, 4:3, blob texture, "
                        f"random similarity, IoU 0.3-0.5), L 16/32/64/128; learned path keeps "
                        f"ceil(0.3 n) keypoints per image by scorer logit",
            "images": 2 * len(pairs), "megapixels": round(mpix, 1),
            "plain_pairs_per_s": round(len(pairs) * 1000.0 / ms_p, 2),
            "learned_pairs_per_s": round(len(pairs) * 1000.0 / ms_l, 2),
            "speedup": round(ms_p / ms_l, 2),
            "plain_ms_per_step": round(ms_p, 2), "learned_ms_per_step": round(ms_l, 2),
            "timing": "graph replays of the preallocated step of each path",
            "plain_ms_per_step_eager": round(out["plain"][2], 2),
            "learned_ms_per_step_eager": round(out["learned"][2], 2),
            "ransac_inliers_plain": int(r[:, 0].sum()), "ransac_inliers_learned": int(r[:, 1].sum()),
            "inlier_retention": round(r[:, 1].sum() / max(r[:, 0].sum(), 1), 4),
            "gt_consistent_plain": int(r[:, 2].sum()), "gt_consistent_learned": int(r[:, 3].sum()),
            "gt_match_retention": round(r[:, 3].sum() / max(r[:, 2].sum(), 1), 4),
            "min_pair_gt_retention": round(float(np.min(r[:, 3] / np.maximum(r[:, 2], 1))), 4),
            "fallbacks": int(r[:, 4].sum()),
            "matches_plain": int(r[:, 5].sum()), "matches_learned": int(r[:, 6].sum()),
            "host_ransac_ms_per_pair": round(1000.0 * t_host, 2),
            "split_bf16x3_certified": {
                "plain_pairs_per_s": round(len(pairs) * 1000.0 / split["plain"][0], 2),
                "learned_pairs_per_s": round(len(pairs) * 1000.0 / split["learned"][0], 2),
                "speedup": round(split["plain"][0] / split["learned"][0], 2),
                "list_agreement_with_fp32": {k: round(v[1], 6) for k, v in split.items()}},
            "weights_sha256": info["sha256"][:16]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(images and match pairs would shard across GPUs with no reduction)",
              file=sys.stderr)
        sys.exit(2)

    # mixed-size pairs for the learned-pruning measurement: rendered by host
    # processes started before this process touches the GPU
    learned_job = pool = None
    if not args.no_learned:
        import multiprocessing as mp
        import synth
        pool = mp.get_context("spawn").Pool(16)
        learned_job = pool.map_async(synth.make_mixed_pair,
                                     synth.mixed_pair_specs(args.learned_pairs), chunksize=1)

    import numpy as np
    import torch

    import synth
    import paper_2405_08578_amd as lp

    dev = torch.device("cuda:0")
    Ls = [16, 32, 64, 128]
    pair = synth.config_pair(1)
    h, w = pair.A.shape
    P = lp.Params(Ls)
    imgs = [torch.from_numpy(pair.A).to(dev), torch.from_numpy(pair.B).to(dev)]
    n_kp = lp.num_keypoints(h, w, P)

    # every buffer allocated once, outside the timed region
    kps = [lp.empty_keypoints(n_kp, dev) for _ in imgs]
    theta = [torch.empty(n_kp, dtype=torch.float32, device=dev) for _ in imgs]
    desc = [torch.empty((n_kp, 128), dtype=torch.float32, device=dev) for _ in imgs]
    ws_d = torch.empty(lp.describe_workspace_size(imgs, P), dtype=torch.uint8, device=dev)
    mp = lp.match_params()
    ws_m = torch.empty(lp.match_workspace_size([n_kp], [n_kp], mp), dtype=torch.uint8, device=dev)
    mout = [{"match": torch.empty(n_kp, dtype=torch.int32, device=dev),
             "d1": torch.empty(n_kp, dtype=torch.float32, device=dev),
             "d2": torch.empty(n_kp, dtype=torch.float32, device=dev)}]
    stream = torch.cuda.current_stream()

    def step():
        lp.detect(imgs, P, out=kps, stream=stream)
        lp.describe(imgs, kps, P, workspace=ws_d, theta=theta, desc=desc, stream=stream)
        lp.match([desc[0]], [desc[1]], workspace=ws_m, out=mout, stream=stream)

    if args.copy_probe_mb > 0:
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if learned_job is not None:
        learned_job.wait()       # no host workers compete with the timed region
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: every launch of the path's kernels is bracketed by HIP
    # events on its own stream (the library's timing facility)
    lp.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt_raw = lp.timing_read()
    lp.timing_enable(False)
    kt = kernel_table(kt_raw, args.steps)

    ms_per_step = 1000.0 * wall / args.steps
    pairs_per_s = 1000.0 / ms_per_step
    mpix = 2 * h * w / 1e6
    dd_ms = sum(kt[k]["ms_per_step"] for k in ("detect", "gradient", "describe") if k in kt)
    m_ms = sum(kt[k]["ms_per_step"] for k in kt if k.startswith("match"))
    flops = 2.0 * n_kp * n_kp * 128
    k_ms = kt["match_fp32"]["ms_per_launch"]
    achieved = flops / (k_ms * 1e-3) / 1e12
    n_match = int((mout[0]["match"] >= 0).sum().item())
    # algorithmic bytes (see the kernel notes): detect reads every pixel and
    # writes 15 B per keypoint slot; the gradient pass reads 1 B and writes 8 B
    # per pixel
    det_bytes = 2 * (h * w + n_kp * 15)
    grad_bytes = 2 * h * w * 9
    # detect + describe against HBM with the algorithmic bytes of both: each
    # image read once, per keypoint slot 16 B of keypoint, 4 B of theta and
    # 512 B of descriptor written (the VALU bounds describe; see the notes)
    dd_bytes = 2 * (h * w + n_kp * (16 + 4 + 512))
    rates = {"detect_describe_algorithmic_GBps": round(dd_bytes / (dd_ms * 1e-3) / 1e9, 1),
             "detect_describe_hbm_frac": round(dd_bytes / (dd_ms * 1e-3) / 1e9 / PEAK_HBM, 4),
             "detect_GBps": round(det_bytes / (kt["detect"]["ms_per_step"] * 1e-3) / 1e9, 1),
             "gradient_GBps": round(grad_bytes / (kt["gradient"]["ms_per_step"] * 1e-3) / 1e9, 1),
             "describe_keypoints_per_s": round(2 * n_kp / (kt["describe"]["ms_per_step"] * 1e-3), 0)}
    # describe against its own roof, the VALU issue rate: the counted VALU
    # instructions of the step over its live event time
    n_valu = describe_valu_instructions()
    if n_valu is not None:
        g = n_valu / (kt["describe"]["ms_per_step"] * 1e-3) / 1e9
        rates["describe_valu"] = {"bound": "alu", "achieved": round(g, 1), "peak": PEAK_VALU_GINSTR,
                                  "unit": "G wave64 VALU instructions/s",
                                  "frac": round(g / PEAK_VALU_GINSTR, 4),
                                  "instructions": n_valu}
    else:
        rates["describe_valu"] = None

    out = {
        "metric": METRIC,
        "value": round(pairs_per_s, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"LP-SIFT plain path on one {w}x{h} uint8 pair (blob texture, "
                               f"random similarity, IoU {pair.iou:.2f}): detect+orient+describe "
                               f"both images, FP32 brute-force match with ratio 0.8",
                   "L": Ls, "descriptors_per_image": n_kp, "desc_dim": 128},
        "detect_describe_mpix_per_s": round(mpix / (dd_ms * 1e-3), 1),
        "detect_describe_ms": round(dd_ms, 4),
        "match_ms": round(m_ms, 4),
        "matches": n_match,
        "kernels": kt,
        "kernel_rates": rates,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4),
                     "traffic": measured_traffic(),
                     "kernel": f"match_topk_f32_kernel, {flops / 1e9:.1f} GFLOP per launch, "
                               f"{k_ms:.4f} ms per launch (HIP events on its stream)"},
    }
    # measured ceilings beside the published ones: a 1 GiB device copy and the
    # matrix-core probes of the four precisions the matchers use
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    copy_ms, _ = timed(lambda: dst.copy_(src), 5, stream)
    out["measured_peaks"] = {
        "hbm_copy_GBps": round(2 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1),
        "mfma_fp32_tflops": round(lp.mfma_probe("fp32"), 1),
        "mfma_bf16_tflops": round(lp.mfma_probe("bf16"), 1),
        "mfma_fp8_tflops": round(lp.mfma_probe("fp8"), 1),
        "mfma_int8_tops": round(lp.mfma_probe("int8"), 1),
        "note": "rates reached by plain copies and register-only MFMA chains on this box; "
                "roofline.peak stays the published figure"}
    del src, dst

    # reduced-precision contractions on the same descriptors (side fields): the
    # split BF16x3 path is certified against the FP32 path, BF16 and FP8 are
    # approximate
    ref = mout[0]["match"].clone()
    lowp = {}
    for prec, name in ((3, "split_bf16x3_certified"), (1, "bf16"), (2, "fp8")):
        mpl = lp.match_params(precision=prec)
        wsl = torch.empty(lp.match_workspace_size([n_kp], [n_kp], mpl), dtype=torch.uint8, device=dev)
        outl = [{k: torch.empty_like(v) for k, v in mout[0].items()}]
        stats = torch.zeros(1, dtype=torch.int32, device=dev)
        call = lambda: lp.match([desc[0]], [desc[1]], precision=prec, workspace=wsl, out=outl,
                                stream=stream, stats=stats)
        for _ in range(max(1, args.warmup)):
            call()
        _, ms = timed(call, args.steps, stream)
        same = (outl[0]["match"] == ref).float().mean().item()
        lowp[name] = {"match_ms": round(ms, 4),
                      "pairs_per_s": round(1000.0 / (dd_ms + ms), 2),
                      "contraction_tflops_equiv": round(flops / (ms * 1e-3) / 1e12, 1),
                      "list_agreement_with_fp32": round(same, 6)}
        if prec == 3:
            lowp[name]["queries_rematched_fp32"] = int(stats.item())
        del wsl, outl
    out["low_precision_match"] = lowp
    # uint8 descriptors (side field): quantise both sets and match them exactly
    # on the int8 matrix cores
    qA = torch.empty((n_kp, 128), dtype=torch.uint8, device=dev)
    qB = torch.empty_like(qA)
    wsu = torch.empty(lp.match_u8_workspace_size(n_kp, n_kp), dtype=torch.uint8, device=dev)
    outu = {k: torch.empty_like(v) for k, v in mout[0].items()}

    def u8_call():
        lp.quantize_u8(desc[0], out=qA, stream=stream)
        lp.quantize_u8(desc[1], out=qB, stream=stream)
        lp.match_u8(qA, qB, workspace=wsu, out=outu, stream=stream)
    for _ in range(max(1, args.warmup)):
        u8_call()
    _, ms = timed(u8_call, args.steps, stream)
    lp.timing_enable(True)
    timed(u8_call, args.steps, stream)
    ku = kernel_table(lp.timing_read(), args.steps)
    lp.timing_enable(False)
    ku_ms = ku["match_u8"]["ms_per_launch"]
    tops = flops / (ku_ms * 1e-3) / 1e12
    out["uint8_exact_match"] = {
        "ms_quantize_and_match": round(ms, 4),
        "pairs_per_s": round(1000.0 / (dd_ms + ms), 2),
        "contraction_ms": round(ku_ms, 4),
        "merge_and_terms_ms": round(ku["match_u8_aux"]["ms_per_step"], 4),
        "contraction_int8_tops": round(tops, 1),
        "frac_of_int8_peak": round(tops / PEAK_INT8_MFMA, 4),
        "list_agreement_with_fp32": round((outu["match"] == ref).float().mean().item(), 6),
        "matches": int((outu["match"] >= 0).sum().item())}
    del qA, qB, wsu, outu

    # multi-orientation rows (side field): secondary orientations >= 0.8 of
    # the highest, up to 4 per keypoint; one untimed FP32 match of the rows
    mo = lp.describe_multi(imgs, kps, P, 4, 0.8, stream=stream)
    wsmo = torch.empty(lp.describe_multi_workspace_size(imgs, P), dtype=torch.uint8, device=dev)
    mo_call = lambda: lp.describe_multi(imgs, kps, P, 4, 0.8, workspace=wsmo, out=mo,
                                        stream=stream)
    for _ in range(max(1, args.warmup)):
        mo_call()
    _, ms_mo = timed(mo_call, args.steps, stream)
    lp.timing_enable(True)
    timed(mo_call, args.steps, stream)
    kmo = kernel_table(lp.timing_read(), args.steps)
    lp.timing_enable(False)
    nr = [int(v) for v in mo["n_rows"].cpu()]
    mm = lp.match([mo["desc"][0][:nr[0]]], [mo["desc"][1][:nr[1]]], stream=stream)[0]
    out["multi_orientation"] = {
        "describe_ms_both_images": round(ms_mo, 4),
        "orientation_pass_ms": kmo["orient_multi"]["ms_per_step"],
        "descriptor_pass_ms": kmo["describe"]["ms_per_step"],
        "single_orientation_describe_ms": round(kt["gradient"]["ms_per_step"] +
                                                kt["describe"]["ms_per_step"], 4),
        "rows_per_keypoint": round(sum(nr) / (2 * n_kp), 4),
        "rows": nr,
        "matches_fp32": int((mm["match"] >= 0).sum().item()),
        "matches_single_orientation": n_match}
    del mo, wsmo, mm
    del kps, theta, desc, ws_d, ws_m, mout
    torch.cuda.empty_cache()

    if not args.no_tiles:
        out["all_pairs_tiles"] = bench_tiles(args, dev)
    if learned_job is not None:
        mixed = learned_job.get()
        pool.close()
        pool.join()
        out["learned_pruning"] = bench_learned(args, dev, mixed)
        del mixed

    if not args.no_cpu_baseline:
        cb = cpu_baseline(pair, Ls, args.cpu_reps)
        out["cpu_baseline"] = {k: (round(v, 6) if isinstance(v, float) else v)
                               for k, v in cb.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
