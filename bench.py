#!/usr/bin/env python3
"""Throughput of the LP-SIFT hot path on one MI355X.

Headline workload: the all-pairs matching of the mosaic (Sec. 4). Nine
shuffled uint8 tiles (2600-2800 x 1600-1800, cut from one 7000x4500 synthetic
world on a 3x3 grid with 25-35 % overlaps) are detected (Eq. 1-2), oriented
and described (Eq. 3-5), and all 36 pairs (i < j) are matched (Eq. 6) with
FP32 matrix-core contractions and the 0.8 ratio test. The whole step (one
detect, one gradient + one describe, three match and three rescore launches,
the candidate split tuned on the device) is captured once in a HIP graph.

One timed step = a 512 MiB device write, which evicts the tiles, keypoints
and descriptors from the L2 caches and the 256 MB Infinity Cache (MALL), then
one graph replay: every step starts cold. value = 36 pairs x K steps / the
wall clock around the K steps (bracketed by device synchronisation); the
write costs ~0.1 ms of each ~140 ms step and is included. The same replays
without the write are reported beside it (warm).

Per-kernel device times come from a separate instrumented pass (eager steps,
each after the same write, with every launch of the path's kernels bracketed
by HIP events on its own stream: the library's timing facility); the roofline
object is computed from it for the dominant kernel, the FP32 contraction.

Side fields: the precision variants of the same step (split BF16x3, certified
exact; BF16 and FP8 approximate; uint8 exact) with their error against the
FP64 oracle on sampled pairs, the mosaic registration and composition, the
single 2600x1600 pair, and learned pruning against the plain path on 32
mixed-size pairs. cpu_baseline: the FP64 oracle on one of the 36 pairs, on
all host threads and on one thread.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--headline-only] [--no-learned]
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s detect+describe; pairs/s matched; learned-pruned vs plain, equal inliers"
PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0           # GB/s
PEAK_INT8_MFMA = 5000.0     # TOP/s, MI355X dense int8 matrix
PEAK_BF16_MFMA = 2500.0     # TFLOP/s dense
PEAK_FP8_MFMA = 5000.0      # TFLOP/s dense
# plain vector ALU: 256 CUs x 64 lanes x 2.4 GHz, one operation per lane per
# clock (an FMA counted once)
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
FLUSH_BYTES = 512 << 20
LS = [16, 32, 64, 128]

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_topk_f32_9_tiles_traffic.md")
MATCH_SRC = os.path.join(ROOT, "paper_2405_08578_amd", "csrc", "match.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline step (tuning, cold and warm replays, the "
                         "instrumented pass): for profiler runs")
    ap.add_argument("--pair-only", action="store_true",
                    help="only the 2600x1600 pair section, printed as one JSON line: for "
                         "profiler runs of detect and describe")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-pruning side measurement (32 mixed-size pairs)")
    ap.add_argument("--learned-pairs", type=int, default=32)
    ap.add_argument("--instrumented-steps", type=int, default=3)
    ap.add_argument("--cpu-reps", type=int, default=2,
                    help="runs of the oracle on the sampled pair on all threads")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the timed region, add 1 to a buffer of this size once "
                         "(untimed): an elementwise kernel of known traffic for calibrating "
                         "HBM counters")
    return ap.parse_args()


# the autotuner's search: candidate-range splits x wavefronts per FP32 workgroup
TUNE_CHUNKS = (2, 4, 6, 8, 12, 16)
TUNE_WAVES = (2, 4, 8)


def log(*a):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


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
    """HBM bytes per launch of the contraction kernel in the headline step,
    from the committed PMC summary, or None when the kernel source changed
    since it was taken."""
    return committed_figure(TRAFFIC_FILE, MATCH_SRC, "match.hip sha256", "traffic bytes per launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


class Flush:
    """A 512 MiB device buffer whose overwrite evicts earlier data from the
    L2 caches and the 256 MB MALL."""

    def __init__(self, dev):
        import torch
        self.buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        self.k = 0

    def __call__(self):
        self.k += 1
        self.buf.fill_(float(self.k & 0xFFFF))


def support_visits(params_L, ws_scale):
    """Algorithmic support of one keypoint per scale: the integer points of
    the descriptor square of side 5 w_s (every pixel with a non-zero
    trilinear weight lies in it; its area, 25 w_s^2) plus the orientation disc
    of radius round(1.5 w_s) (integer points counted exactly)."""
    out = []
    for ws in ws_scale:
        R = int(math.floor(1.5 * ws + 0.5))
        disc = sum(2 * math.isqrt(R * R - dx * dx) + 1 for dx in range(-R, R + 1))
        out.append(25.0 * ws * ws + disc)
    return out


def subregion_sides(Ls, d=4):
    """w_s per scale with the default beta0 = (1/d) sqrt(Lmin / Lmax) (Eq. 3-4)."""
    b0 = (1.0 / d) * math.sqrt(min(Ls) / max(Ls))
    return [b0 * (L / max(Ls)) ** -0.5 * L for L in Ls]


def pair_geometry(tiles):
    """Edge neighbours and disjoint pairs of the shuffled 3x3 tile set."""
    pos = [(int(g) // 3, int(g) % 3) for g in tiles.order]
    nb, far = [], []
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            dy, dx = abs(pos[i][0] - pos[j][0]), abs(pos[i][1] - pos[j][1])
            if dy + dx == 1:
                nb.append((i, j))
            elif max(dy, dx) >= 2:
                far.append((i, j))
    return nb, far


# ----------------------------------------------------------------- headline --

def headline(args, dev, tiles, flush, out):
    """The 9-tile all-pairs step (FP32 match), tuned, graph-replayed cold and
    warm, then one instrumented pass. Fills `out` and returns the AllPairs
    object (kept for the side measurements) and its tuning."""
    import torch
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd.allpairs import AllPairs

    P = lp.Params(LS)
    imgs = [torch.from_numpy(t).to(dev) for t in tiles.images]
    stream = torch.cuda.current_stream()
    n_kp = [lp.num_keypoints(t.shape[0], t.shape[1], P) for t in imgs]

    # tune the candidate-range split of the FP32 and split matchers on the
    # real descriptor sets (device-timed, outside every timed region)
    ap = AllPairs(imgs, P, precision=0)
    ap.run()
    torch.cuda.synchronize()
    A = [ap.desc[i] for i, _ in ap.pairs]
    B = [ap.desc[j] for _, j in ap.pairs]
    tunes = {prec: lp.match_tune(A, B, precision=prec, candidates=TUNE_CHUNKS, waves=TUNE_WAVES,
                                 reps=1)
             for prec in (0, 3)}
    log("tuned:", {p: (t["b_chunks"], t["qblock_waves"]) for p, t in tunes.items()})
    del A, B, ap
    torch.cuda.empty_cache()

    ap = AllPairs(imgs, P, precision=0, b_chunks=tunes[0]["b_chunks"],
                  qblock_waves=tunes[0]["qblock_waves"])
    ap.capture()
    for _ in range(args.warmup):
        flush()
        ap.replay()
    torch.cuda.synchronize()

    if args.copy_probe_mb > 0:
        # an elementwise kernel that reads and writes exactly this many bytes
        # (a plain copy_ would go to the DMA engines, not a kernel)
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # timed region: K cold steps (write, replay); events around each replay
    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        flush()
        ev[k][0].record(stream)
        ap.replay()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    replay_ms = sorted(a.elapsed_time(b) for a, b in ev)
    ms_per_step = 1000.0 * wall / K

    warm_ms, _ = timed(ap.replay, K, stream)
    flush_ms, flush_ev = timed(flush, K, stream)

    # instrumented pass: eager cold steps with per-launch events
    n_i = max(1, args.instrumented_steps)
    lp.timing_enable(True)
    for _ in range(n_i):
        flush()
        ap.run()
    torch.cuda.synchronize()
    kt = kernel_table(lp.timing_read(), n_i)
    lp.timing_enable(False)

    pixels = sum(t.shape[0] * t.shape[1] for t in tiles.images)
    flops = sum(2.0 * n_kp[i] * n_kp[j] * 128 for i, j in ap.pairs)
    dd_ms = sum(kt[k]["ms_per_step"] for k in ("detect", "gradient", "describe") if k in kt)
    m_ms = sum(kt[k]["ms_per_step"] for k in kt if k.startswith("match"))
    mk = kt["match_fp32"]
    launches = mk["launches_per_step"]
    flops_per_launch = flops / launches
    achieved = flops_per_launch / (mk["ms_per_launch"] * 1e-3) / 1e12
    n_match = int(sum(int((o["match"] >= 0).sum().item()) for o in ap.out))

    # algorithmic bytes: detect reads every pixel and writes 15 B per slot;
    # the gradient pass reads 1 B and writes 8 B per pixel; detect+describe
    # as a whole reads each image once and writes per slot 16 B of keypoint,
    # 4 B of theta and 512 B of descriptor
    n_slots = sum(n_kp)
    det_bytes = pixels + 15 * n_slots
    grad_bytes = 9 * pixels
    dd_bytes = pixels + n_slots * (16 + 4 + 512)
    ws_s = subregion_sides(LS)
    per_kp = support_visits(LS, ws_s)
    visits = 0.0
    for t in tiles.images:
        h, w = t.shape
        for s, L in enumerate(LS):
            visits += 2 * math.ceil(h / L) * math.ceil(w / L) * per_kp[s]
    desc_s = kt["describe"]["ms_per_step"] * 1e-3 + kt["gradient"]["ms_per_step"] * 1e-3
    ops_per_visit = 25.0
    valu_t = visits * ops_per_visit / desc_s / 1e12
    rates = {
        "detect_GBps": round(det_bytes / (kt["detect"]["ms_per_step"] * 1e-3) / 1e9, 1),
        "detect_hbm_frac": round(det_bytes / (kt["detect"]["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM, 4),
        "gradient_GBps": round(grad_bytes / (kt["gradient"]["ms_per_step"] * 1e-3) / 1e9, 1),
        "describe_keypoints_per_s": round(n_slots / (kt["describe"]["ms_per_step"] * 1e-3), 0),
        "detect_describe_algorithmic_GBps": round(dd_bytes / (dd_ms * 1e-3) / 1e9, 1),
        "detect_describe_hbm_frac": round(dd_bytes / (dd_ms * 1e-3) / 1e9 / PEAK_HBM, 4),
        "describe_alu": {
            "bound": "alu", "achieved": round(valu_t, 2), "peak": round(PEAK_VALU_TOPS, 2),
            "unit": "T lane-ops/s", "frac": round(valu_t / PEAK_VALU_TOPS, 4),
            "work": f"{visits / 1e6:.1f} M support visits per step (descriptor square of side "
                    f"5 w_s + orientation disc per keypoint) x {ops_per_visit:.0f} operations "
                    f"per visit, over the gradient + describe time"},
    }

    out.update({
        "metric": METRIC,
        "value": round(36 * 1000.0 / ms_per_step, 3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "LP-SIFT all-pairs step: 9 shuffled uint8 tiles 2600-2800 x "
                               "1600-1800 cut from a 7000x4500 synthetic blob world (3x3 grid, "
                               "25-35 % overlaps, per-tile similarity and gain); detect+orient+"
                               "describe all tiles, FP32 brute-force match of all 36 pairs with "
                               "ratio 0.8; one HIP-graph replay per step, MALL flushed (512 MiB "
                               "written) before each step",
                   "tiles": [list(t.shape) for t in tiles.images], "pairs": 36, "L": LS,
                   "descriptors": n_slots, "desc_dim": 128,
                   "b_chunks": tunes[0]["b_chunks"], "qblock_waves": tunes[0]["qblock_waves"]},
        "timing": {"cold_ms_per_step": round(ms_per_step, 4),
                   "replay_event_ms_median": round(replay_ms[len(replay_ms) // 2], 4),
                   "replay_event_ms_min_max": [round(replay_ms[0], 4), round(replay_ms[-1], 4)],
                   "warm_ms_per_step": round(warm_ms, 4),
                   "warm_pairs_per_s": round(36 * 1000.0 / warm_ms, 3),
                   "flush_ms": round(flush_ev, 4),
                   "instrumented_pass": f"{n_i} eager steps, each after the same 512 MiB write"},
        "detect_describe_mpix_per_s": round(pixels / 1e6 / (dd_ms * 1e-3), 1),
        "detect_describe_ms": round(dd_ms, 4),
        "match_ms": round(m_ms, 4),
        "matches": n_match,
        "kernels": kt,
        "kernel_rates": rates,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4),
                     "traffic": measured_traffic(),
                     "kernel": f"match_topk_f32_kernel: {launches:g} launch(es) per step "
                               f"(up to 36 pairs per launch), {flops / 1e12:.3f} TFLOP per step = "
                               f"{flops_per_launch / 1e9:.1f} GFLOP per launch on average, "
                               f"{mk['ms_per_launch']:.4f} ms per launch (HIP events on its "
                               f"stream, instrumented pass)"},
    })
    tune = {"fp32": tunes[0], "split": tunes[3]}
    return ap, imgs, P, n_kp, flops, tune


# --------------------------------------------------- oracle error (cfg3) --

def oracle_errors(ap_desc, pairs, lists):
    """Error of each precision's lists and distances against the FP64 oracle
    matcher run on the same FP32 descriptors, on the sampled pairs.
    lists[name][p] = host dict (match, d1, d2) of sampled pair p."""
    import numpy as np
    import oracle
    res = {name: {"queries": 0, "agree_all": 0, "agree_outside_band": 0, "outside_band": 0,
                  "recall_j1": 0, "recall_j1_j2": 0, "d1_rel_err_max_recalled": 0.0,
                  "d1_rel_err_median": []} for name in lists}
    for p, (i, j) in enumerate(pairs):
        A = ap_desc[i].cpu().numpy().astype(np.float64)
        B = ap_desc[j].cpu().numpy().astype(np.float64)
        o = oracle.match(A, B)
        d1o, d2o = o["d1"], o["d2"]
        with np.errstate(divide="ignore", invalid="ignore"):
            marg = np.minimum(np.abs(d1o / d2o - 0.8), (d2o - d1o) / np.maximum(d1o, 1e-300))
        safe = marg > 1e-6
        tol = lambda d: 2e-6 * d + 1e-6
        for name, per in lists.items():
            g = per[p]
            r = res[name]
            rec1 = np.abs(g["d1"] - d1o) <= tol(d1o)
            rec12 = rec1 & (np.abs(g["d2"] - d2o) <= tol(d2o))
            r["queries"] += len(A)
            r["agree_all"] += int((g["match"] == o["match"]).sum())
            r["outside_band"] += int(safe.sum())
            r["agree_outside_band"] += int((g["match"][safe] == o["match"][safe]).sum())
            r["recall_j1"] += int(rec1.sum())
            r["recall_j1_j2"] += int(rec12.sum())
            rel = np.abs(g["d1"] - d1o) / np.maximum(d1o, 1e-30)
            if rec1.any():
                r["d1_rel_err_max_recalled"] = max(r["d1_rel_err_max_recalled"],
                                                   float(rel[rec1].max()))
            r["d1_rel_err_median"].append(float(np.median(rel)))
    out = {}
    for name, r in res.items():
        q = max(r["queries"], 1)
        out[name] = {"list_agreement_with_fp64": round(r["agree_all"] / q, 6),
                     "list_agreement_outside_1e-6_band": round(
                         r["agree_outside_band"] / max(r["outside_band"], 1), 6),
                     "recall_j1": round(r["recall_j1"] / q, 6),
                     "recall_j1_j2": round(r["recall_j1_j2"] / q, 6),
                     "d1_rel_err_max_recalled": float(f"{r['d1_rel_err_max_recalled']:.3g}"),
                     "d1_rel_err_median": float(f"{np.median(r['d1_rel_err_median']):.3g}")}
    return out


def precision_variants(args, dev, tiles, imgs, P, n_kp, flops, tune, ref_lists, ap_desc):
    """The same 9-tile step with the other matchers, graph-replayed, and the
    error of every matcher against the FP64 oracle on sampled pairs."""
    import numpy as np
    import torch
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd.allpairs import AllPairs

    stream = torch.cuda.current_stream()
    steps = max(2, args.steps // 2)
    nb, far = pair_geometry(tiles)
    sample = [nb[0], far[0]] if far else [nb[0]]
    ap_pairs = [(i, j) for i in range(9) for j in range(i + 1, 9)]
    sidx = [ap_pairs.index(p) for p in sample]
    sampled = {"fp32": [ref_lists[k] for k in sidx]}
    variants = {}
    peaks = {3: PEAK_BF16_MFMA, 1: PEAK_BF16_MFMA, 2: PEAK_FP8_MFMA}
    # the quantised matchers' candidate split, tuned like the FP32 one
    A = [ap_desc[i] for i, _ in ap_pairs]
    B = [ap_desc[j] for _, j in ap_pairs]
    lp_tune = {prec: lp.match_tune(A, B, precision=prec, candidates=TUNE_CHUNKS, reps=1)
               for prec in (1, 2)}
    del A, B
    for prec, name in ((3, "split_bf16x3_certified"), (1, "bf16"), (2, "fp8")):
        bc = tune["split"]["b_chunks"] if prec == 3 else lp_tune[prec]["b_chunks"]
        qw = tune["split"]["qblock_waves"] if prec == 3 else 0
        ap = AllPairs(imgs, P, precision=prec, b_chunks=bc, qblock_waves=qw)
        ap.capture()
        for _ in range(max(1, args.warmup)):
            ap.replay()
        wall, _ = timed(ap.replay, steps, stream)
        lp.timing_enable(True)
        ap.run()
        torch.cuda.synchronize()
        kt = kernel_table(lp.timing_read(), 1)
        lp.timing_enable(False)
        lists = [{k: v.cpu().numpy() for k, v in o.items()} for o in ap.out]
        same = sum(int((a["match"] == b["match"]).sum()) for a, b in zip(lists, ref_lists))
        key = "match_split" if prec == 3 else "match_lowp"
        v = {"ms_per_step_graph": round(wall, 3), "pairs_per_s": round(36 * 1000.0 / wall, 3),
             "b_chunks": bc, "kernels": kt,
             "list_agreement_with_fp32": round(same / sum(len(m["match"]) for m in lists), 6)}
        if key in kt:
            tf = flops / (kt[key]["ms_per_step"] * 1e-3) / 1e12
            v["contraction_tflops_equiv"] = round(tf, 1)
            if prec in (1, 2):
                v["frac_of_peak"] = round(tf / peaks[prec], 4)
        if prec == 3:
            v["queries_rematched_fp32"] = int(ap.stats.item())
        variants[name] = v
        sampled[name] = [lists[k] for k in sidx]
        del ap
        torch.cuda.empty_cache()

    # exact uint8 variant (quantise all 9 sets, integer match of every pair)
    ap = AllPairs(imgs, P, u8=True)
    ap.capture()
    for _ in range(max(1, args.warmup)):
        ap.replay()
    wall, _ = timed(ap.replay, steps, stream)
    lp.timing_enable(True)
    ap.run()
    torch.cuda.synchronize()
    kt = kernel_table(lp.timing_read(), 1)
    lp.timing_enable(False)
    same = sum(int((o["match"].cpu().numpy() == r["match"]).sum())
               for o, r in zip(ap.out, ref_lists))
    k_ms = kt["match_u8"]["ms_per_step"]
    variants["uint8_exact"] = {
        "ms_per_step_graph": round(wall, 3), "pairs_per_s": round(36 * 1000.0 / wall, 3),
        "kernels": kt, "contraction_int8_tops": round(flops / (k_ms * 1e-3) / 1e12, 1),
        "frac_of_int8_peak": round(flops / (k_ms * 1e-3) / 1e12 / PEAK_INT8_MFMA, 4),
        "matches": int(sum(int((o["match"] >= 0).sum().item()) for o in ap.out)),
        "list_agreement_with_fp32": round(same / sum(len(m["match"]) for m in ref_lists), 6)}
    del ap
    torch.cuda.empty_cache()

    errs = oracle_errors(ap_desc, sample, sampled)
    return {"variants": variants,
            "error_vs_fp64_oracle": {
                "pairs": [list(p) for p in sample],
                "what": "the FP64 oracle matcher on the step's own FP32 descriptors of one "
                        "neighbouring and one disjoint tile pair; recall = the reported d1 "
                        "(d1 and d2) equal the exact FP64 distances to 2e-6 relative + 1e-6; "
                        "the band = queries within 1e-6 of a decision boundary",
                "by_precision": errs}}


# ---------------------------------------------------- mosaic registration --

def registration(args, dev, tiles, imgs, P, tune):
    """Mosaic registration: the FP32 all-pairs step plus the batched GPU
    RANSAC of all 36 pairs in one graph, the rounds of Sec. 4 on the host,
    then warp and blend of the registered tiles."""
    import numpy as np
    import torch
    import synth
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd import mosaic as M
    from paper_2405_08578_amd.allpairs import AllPairs

    stream = torch.cuda.current_stream()
    steps = max(2, args.steps // 4)
    u = torch.from_numpy(synth.ransac_uniforms(16384, np.random.default_rng(11))).to(dev)
    ap = AllPairs(imgs, P, precision=0, b_chunks=tune["fp32"]["b_chunks"],
                  qblock_waves=tune["fp32"]["qblock_waves"], ransac_uniforms=u)
    ap.capture()
    for _ in range(max(1, args.warmup)):
        ap.replay()
    wall, _ = timed(ap.replay, steps, stream)
    lp.timing_enable(True)
    ap.run()
    torch.cuda.synchronize()
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
    # joint refinement of the placements over every stitchable pair's inliers
    t1 = time.perf_counter()
    kps = [{k: v.cpu().numpy() for k, v in kp.items()} for kp in ap.kps]
    corr = M.correspondences(ap.pairs, kps, [t.cpu().numpy() for t in ap.ransac["slotA"]],
                             [t.cpu().numpy() for t in ap.ransac["slotB"]],
                             [t.cpu().numpy() for t in ap.ransac["inlier"]], st, W)
    G_ref, rinfo = M.refine(reg["G"], corr, ref)
    refine_ms = 1000.0 * (time.perf_counter() - t1)
    seams_r = M.seam_errors(G_ref, G_true, [t.shape for t in tiles.images])
    res = {
        "what": "9 tiles: detect+describe, FP32 match of 36 pairs, GPU RANSAC (16384 "
                "hypotheses per pair, 3 px) in one graph replay; then H_M rounds on the host",
        "ms_per_step_graph": round(wall, 3), "host_rounds_ms": round(host_ms, 3),
        "ransac_ms": kt.get("ransac", {}).get("ms_per_step"),
        "registered": len(imgs) - len(reg["unregistered"]),
        "stitchable_pairs": int((W > 0).sum() // 2),
        "inliers_on_links": [int(W[a, b]) for a, b in reg["links"]],
        "max_link_seam_px": round(max(link), 3) if link else None,
        "max_overlap_seam_px": round(max(seams.values()), 3) if seams else None,
        "refined": {"max_overlap_seam_px": round(max(seams_r.values()), 3) if seams_r else None,
                    "rms_px_before": round(rinfo["rms_before"], 3),
                    "rms_px_after": round(rinfo["rms_after"], 3), "iters": rinfo["iters"],
                    "host_ms": round(refine_ms, 1),
                    "what": "Levenberg-Marquardt over all stitchable pairs' RANSAC inliers, "
                            "reference fixed"},
        "paper_context": "the paper stitches nine images over 2600x1600 in 158.94 s "
                         "(MATLAB on an Intel i9-12900, including warping and blending; "
                         "here they are the warp_blend figures)"}
    idx = [k for k in range(len(imgs)) if G_ref[k] is not None]
    Gs = [G_ref[k] for k in idx]
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
    res["warp_blend"] = {
        "canvas": [cw, ch], "images": len(wimgs),
        "ms": round(wms, 4), "kernel_ms": kw["warp"]["ms_per_launch"],
        "algorithmic_GBps": round(wbytes / (kw["warp"]["ms_per_launch"] * 1e-3) / 1e9, 1),
        "covered_share": round(both.float().mean().item(), 4),
        "mean_abs_diff_vs_true_transforms": round(diff.mean().item(), 3),
        "end_to_end_ms": round(wall + host_ms + wms, 3)}
    del canvas, count, est, est_count, ap
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------ the single 2600x1600 pair --

def single_pair(args, dev, flush):
    """One 2600x1600 pair (the two-image workload): detect + describe both
    images and match, eager with preallocated buffers, cold (after the same
    512 MiB write) per step; the other matchers and variants on its
    descriptors."""
    import torch
    import synth
    import paper_2405_08578_amd as lp

    pair = synth.config_pair(1)
    h, w = pair.A.shape
    P = lp.Params(LS)
    imgs = [torch.from_numpy(pair.A).to(dev), torch.from_numpy(pair.B).to(dev)]
    n_kp = lp.num_keypoints(h, w, P)
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

    for _ in range(args.warmup):
        step()
    steps = args.steps
    e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
         for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        flush()
        e[k][0].record(stream)
        step()
        e[k][1].record(stream)
    torch.cuda.synchronize()
    cold = sorted(a.elapsed_time(b) for a, b in e)
    warm_ms, warm_ev = timed(step, steps, stream)
    lp.timing_enable(True)
    for _ in range(steps):
        flush()
        step()
    torch.cuda.synchronize()
    kt = kernel_table(lp.timing_read(), steps)
    lp.timing_enable(False)
    flops = 2.0 * n_kp * n_kp * 128
    dd_ms = sum(kt[k]["ms_per_step"] for k in ("detect", "gradient", "describe") if k in kt)
    k_ms = kt["match_fp32"]["ms_per_launch"]
    cold_ms = cold[len(cold) // 2]
    res = {"workload": f"one {w}x{h} uint8 pair (blob texture, random similarity, IoU "
                       f"{pair.iou:.2f}): detect+orient+describe both images, FP32 match "
                       f"with ratio 0.8, eager launches into preallocated buffers",
           "descriptors_per_image": n_kp,
           "cold_ms_per_step_event_median": round(cold_ms, 4),
           "pairs_per_s_cold": round(1000.0 / cold_ms, 3),
           "warm_ms_per_step_event": round(warm_ev, 4),
           "pairs_per_s_warm": round(1000.0 / warm_ev, 3),
           "detect_describe_ms": round(dd_ms, 4),
           "detect_describe_mpix_per_s": round(2 * h * w / 1e6 / (dd_ms * 1e-3), 1),
           "contraction_ms": k_ms,
           "contraction_tflops": round(flops / (k_ms * 1e-3) / 1e12, 2),
           "contraction_frac_of_peak": round(flops / (k_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA, 4),
           "matches": int((mout[0]["match"] >= 0).sum().item()),
           "kernels": kt}

    ref = mout[0]["match"].clone()
    lowp = {}
    for prec, name in ((3, "split_bf16x3_certified"), (1, "bf16"), (2, "fp8")):
        mpl = lp.match_params(precision=prec)
        wsl = torch.empty(lp.match_workspace_size([n_kp], [n_kp], mpl), dtype=torch.uint8,
                          device=dev)
        outl = [{k: torch.empty_like(v) for k, v in mout[0].items()}]
        stats = torch.zeros(1, dtype=torch.int32, device=dev)
        call = lambda: lp.match([desc[0]], [desc[1]], precision=prec, workspace=wsl, out=outl,
                                stream=stream, stats=stats)
        for _ in range(max(1, args.warmup)):
            call()
        _, ms = timed(call, args.steps, stream)
        lowp[name] = {"match_ms": round(ms, 4),
                      "contraction_tflops_equiv": round(flops / (ms * 1e-3) / 1e12, 1),
                      "list_agreement_with_fp32": round(
                          (outl[0]["match"] == ref).float().mean().item(), 6)}
        if prec == 3:
            lowp[name]["queries_rematched_fp32"] = int(stats.item())
        del wsl, outl
    res["low_precision_match"] = lowp

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
    res["uint8_exact_match"] = {
        "ms_quantize_and_match": round(ms, 4), "contraction_ms": round(ku_ms, 4),
        "contraction_int8_tops": round(tops, 1), "frac_of_int8_peak": round(tops / PEAK_INT8_MFMA, 4),
        "list_agreement_with_fp32": round((outu["match"] == ref).float().mean().item(), 6),
        "matches": int((outu["match"] >= 0).sum().item())}
    del qA, qB, wsu, outu

    mo = lp.describe_multi(imgs, kps, P, 4, 0.8, stream=stream)
    wsmo = torch.empty(lp.describe_multi_workspace_size(imgs, P), dtype=torch.uint8, device=dev)
    mo_call = lambda: lp.describe_multi(imgs, kps, P, 4, 0.8, workspace=wsmo, out=mo,
                                        stream=stream)
    for _ in range(max(1, args.warmup)):
        mo_call()
    _, ms_mo = timed(mo_call, args.steps, stream)
    nr = [int(v) for v in mo["n_rows"].cpu()]
    mm = lp.match([mo["desc"][0][:nr[0]]], [mo["desc"][1][:nr[1]]], stream=stream)[0]
    res["multi_orientation"] = {
        "describe_ms_both_images": round(ms_mo, 4),
        "rows_per_keypoint": round(sum(nr) / (2 * n_kp), 4), "rows": nr,
        "matches_fp32": int((mm["match"] >= 0).sum().item())}
    del mo, wsmo, mm, kps, theta, desc, ws_d, ws_m, mout
    torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------- learned path --

def bench_learned(args, dev, pairs):
    """Learned pruning vs the plain path on mixed-size pairs (1024x768 ..
    4000x3000): GPU pairs/s of both paths over all pairs at once (every image
    in the same detect/score/prune/describe calls, all pairs in one match
    call; inputs resident; graph replays), then host RANSAC on both results.
    Retention is measured per pair on the plain path's RANSAC inliers: the
    share of its (slot in A, slot in B) inlier pairs that are also inliers of
    the learned path."""
    import numpy as np
    import torch
    import paper_2405_08578_amd as lp
    from paper_2405_08578_amd import learned as L

    w, info = L.load_weights(L.DEFAULT_WEIGHTS, dev)
    P = lp.Params(LS)
    imgs = [[torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev)] for p in pairs]
    mpix = sum(2 * p.A.size for p in pairs) / 1e6
    steps = max(1, min(3, args.steps // 5))

    def timed_path(bp):
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

    def run(weights, num=3, den=10):
        bp = L.BatchPath(imgs, P, weights=weights, num=num, den=den)
        g_ms, e_ms = timed_path(bp)
        res = bp.results()
        del bp
        return g_ms, res, e_ms

    out = {"plain": run(None), "learned": run(w)}
    torch.cuda.empty_cache()
    rows, kept = [], []
    t0 = time.perf_counter()
    plain = [L.finish(out["plain"][1][k], seed=k, H_true=p.H) for k, p in enumerate(pairs)]
    for k, p in enumerate(pairs):
        pl = plain[k]
        le = L.finish(out["learned"][1][k], seed=k, H_true=p.H)
        fb = L.needs_fallback(le)
        if fb:
            le = pl
        kept.append(L.inlier_retention(pl, le))
        rows.append((pl["inliers"], le["inliers"], pl["gt_consistent"], le["gt_consistent"], fb,
                     pl["matches"], le["matches"]))
    t_host = (time.perf_counter() - t0) / (2 * len(pairs))
    r = np.array(rows, dtype=np.float64)
    kept = np.array(kept, dtype=np.float64)          # [pairs, 2]: kept, plain inliers
    per_pair = kept[:, 0] / np.maximum(kept[:, 1], 1)
    ms_p, ms_l = out["plain"][0], out["learned"][0]

    # the same measurement at larger keep fractions (retention against cost)
    curve = []
    for num, den in ((7, 20), (2, 5)):
        g_ms, res, _ = run(w, num, den)
        kk = []
        for k, p in enumerate(pairs):
            le = L.finish(res[k], seed=k)
            kk.append(L.inlier_retention(plain[k], plain[k] if L.needs_fallback(le) else le))
        kk = np.array(kk, dtype=np.float64)
        curve.append({"keep": f"{num}/{den}", "learned_pairs_per_s": round(len(pairs) * 1000.0 / g_ms, 2),
                      "speedup": round(ms_p / g_ms, 2),
                      "inlier_retention": round(float(kk[:, 0].sum() / max(kk[:, 1].sum(), 1)), 4),
                      "inlier_retention_min_pair":
                          round(float((kk[:, 0] / np.maximum(kk[:, 1], 1)).min()), 4)})
        del res
        torch.cuda.empty_cache()
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
            "inlier_retention": round(float(kept[:, 0].sum() / max(kept[:, 1].sum(), 1)), 4),
            "inlier_retention_min_pair": round(float(per_pair.min()), 4),
            "inlier_retention_what": "plain-path RANSAC inliers (slot in A, slot in B) that "
                                     "are also learned-path inliers (after fallback), summed "
                                     "over pairs; min_pair = the lowest pair's share",
            "ransac_inliers_plain": int(r[:, 0].sum()), "ransac_inliers_learned": int(r[:, 1].sum()),
            "inlier_count_ratio": round(r[:, 1].sum() / max(r[:, 0].sum(), 1), 4),
            "gt_consistent_plain": int(r[:, 2].sum()), "gt_consistent_learned": int(r[:, 3].sum()),
            "gt_match_retention": round(r[:, 3].sum() / max(r[:, 2].sum(), 1), 4),
            "min_pair_gt_retention": round(float(np.min(r[:, 3] / np.maximum(r[:, 2], 1))), 4),
            "fallbacks": int(r[:, 4].sum()),
            "matches_plain": int(r[:, 5].sum()), "matches_learned": int(r[:, 6].sum()),
            "host_ransac_ms_per_pair": round(1000.0 * t_host, 2),
            "ransac": f"{L.RANSAC_ITERS} hypotheses per pair, then least-squares rounds over the "
                      f"inliers until the inlier set is unchanged (at most {L.REFINE_ROUNDS})",
            "keep_curve": curve,
            "weights_sha256": info["sha256"][:16]}


# ------------------------------------------------------------- CPU oracle --

def cpu_baseline(tiles, pair, reps=2):
    """The FP64 oracle on one pair of the headline step (tiles i and j):
    detect+orient+describe both tiles and the brute-force matcher over every
    query, on all OpenMP threads (`reps` runs, the median per pair); and on
    one thread with the matcher run on every 48th query and scaled to all."""
    import numpy as np
    import oracle
    i, j = pair
    A, B = tiles.images[i], tiles.images[j]
    gomp = ctypes.CDLL("libgomp.so.1")
    n_all = int(gomp.omp_get_max_threads())
    times, t_dd, t_m = [], [], []
    nA = nB = 0
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, dA = oracle.features(A, LS)
        _, _, dB = oracle.features(B, LS)
        t1 = time.perf_counter()
        oracle.match(dA, dB)
        t2 = time.perf_counter()
        t_dd.append(t1 - t0)
        t_m.append(t2 - t1)
        times.append(t2 - t0)
        nA, nB = len(dA), len(dB)
    t_pair = float(np.median(times))
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        _, _, dA = oracle.features(A, LS)
        _, _, dB = oracle.features(B, LS)
        t1 = time.perf_counter()
        sel = np.arange(0, len(dA), 48)
        oracle.match(dA[sel], dB)
        t2 = time.perf_counter()
    finally:
        gomp.omp_set_num_threads(n_all)
    t1_pair = (t1 - t0) + (t2 - t1) * len(dA) / len(sel)
    return {"value": round(1.0 / t_pair, 6), "unit": "pairs/s", "cores": n_all, "kind": "oracle",
            "sample": (f"FP64 oracle on pair ({i}, {j}) of the 36 (tiles {A.shape[1]}x{A.shape[0]} "
                       f"and {B.shape[1]}x{B.shape[0]}), {reps} runs on {n_all} threads: "
                       f"detect+describe both tiles (median {np.median(t_dd):.2f} s) + "
                       f"brute-force match of all {nA} queries vs {nB} (median "
                       f"{np.median(t_m):.2f} s); value = 1 / seconds per pair"),
            "seconds_per_pair": round(t_pair, 3),
            "cpu_model": cpu_model(),
            "one_thread": {"value": round(1.0 / t1_pair, 6), "unit": "pairs/s", "cores": 1,
                           "seconds_per_pair": round(t1_pair, 2),
                           "sample": (f"same pair on 1 thread: detect+describe both tiles "
                                      f"{t1 - t0:.2f} s + match of {len(sel)} of {len(dA)} "
                                      f"queries (every 48th) {t2 - t1:.2f} s, scaled to all")}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: liblpsift has no multi-GPU path (images and "
              "match pairs would shard across GPUs with no reduction)", file=sys.stderr)
        sys.exit(2)

    # mixed-size pairs for the learned-pruning measurement: rendered by host
    # processes started before this process touches the GPU
    if args.pair_only:
        import torch
        dev = torch.device("cuda:0")
        print(json.dumps({"pair_2600x1600": single_pair(args, dev, Flush(dev))}), flush=True)
        return

    learned_job = pool = None
    if not (args.no_learned or args.headline_only):
        import multiprocessing as mp
        import synth
        pool = mp.get_context("spawn").Pool(16)
        learned_job = pool.map_async(synth.make_mixed_pair,
                                     synth.mixed_pair_specs(args.learned_pairs), chunksize=1)

    import torch
    import synth
    import paper_2405_08578_amd as lp

    dev = torch.device("cuda:0")
    tiles = synth.make_tiles()
    log("tiles rendered")
    if learned_job is not None:
        learned_job.wait()       # no host workers compete with the timed region
        log("mixed-size pairs rendered")
    flush = Flush(dev)
    out = {}
    ap, imgs, P, n_kp, flops, tune = headline(args, dev, tiles, flush, out)
    log(f"headline: {out['value']} pairs/s, {out['ms_per_step']} ms per step")
    ref_lists = [{k: v.cpu().numpy() for k, v in o.items()} for o in ap.out]
    ap_desc = ap.desc
    out["tuning"] = {"fp32_b_chunks": tune["fp32"]["b_chunks"],
                     "fp32_qblock_waves": tune["fp32"]["qblock_waves"],
                     "split_b_chunks": tune["split"]["b_chunks"],
                     "split_qblock_waves": tune["split"]["qblock_waves"],
                     "candidates": tune["fp32"]["candidates"], "waves": tune["fp32"]["waves"],
                     "fp32_ms": [[round(v, 2) for v in row] for row in tune["fp32"]["ms"]],
                     "split_ms": [[round(v, 2) for v in row] for row in tune["split"]["ms"]]}
    if not args.headline_only:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        copy_ms, _ = timed(lambda: dst.copy_(src), 5, torch.cuda.current_stream())
        out["measured_peaks"] = {
            "hbm_copy_GBps": round(2 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1),
            "mfma_fp32_tflops": round(lp.mfma_probe("fp32"), 1),
            "mfma_bf16_tflops": round(lp.mfma_probe("bf16"), 1),
            "mfma_fp8_tflops": round(lp.mfma_probe("fp8"), 1),
            "mfma_int8_tops": round(lp.mfma_probe("int8"), 1),
            "note": "rates reached by plain copies and register-only MFMA chains on this box; "
                    "roofline.peak stays the published figure"}
        del src, dst
        descs = [d.clone() for d in ap_desc]
        del ap
        torch.cuda.empty_cache()
        out["precision_variants"] = precision_variants(args, dev, tiles, imgs, P, n_kp, flops,
                                                       tune, ref_lists, descs)
        del descs
        log("precision variants done")
        out["registration"] = registration(args, dev, tiles, imgs, P, tune)
        log("registration done")
        out["pair_2600x1600"] = single_pair(args, dev, flush)
        log("single pair done")
    else:
        del ap
    del imgs
    torch.cuda.empty_cache()
    if learned_job is not None:
        mixed = learned_job.get()
        pool.close()
        pool.join()
        out["learned_pruning"] = bench_learned(args, dev, mixed)
        del mixed
        log("learned pruning done")

    if not (args.no_cpu_baseline or args.headline_only):
        nb, _ = pair_geometry(tiles)
        out["cpu_baseline"] = cpu_baseline(tiles, nb[0], args.cpu_reps)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
