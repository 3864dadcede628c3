#!/usr/bin/env python3
"""Throughput of the LP-SIFT hot path on one MI355X.

One step = detect + orient + describe both images of a 2600x1600 uint8 pair
(L = 16, 32, 64, 128) and match every reference descriptor against the
registered set with the 0.8 ratio test: the whole GPU hot path for one pair,
inputs resident in HBM before the timed region.

Prints ONE JSON line: value = pairs/s; detect+describe Mpix/s as a side field;
a roofline object for the dominant kernel (the FP32 matrix-core contraction of
the matcher) from HIP events recorded around every matcher call on the stream
the kernels run on; and the FP64 oracle timed on a bounded sample on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=12288,
                    help="reference descriptors in the oracle's timed match sample")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before warm-up, copy a buffer of this size once (untimed): a plain "
                         "copy kernel of known traffic for calibrating HBM counters")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_topk_f32_2600x1600_pair_traffic.md")
MATCH_SRC = os.path.join(ROOT, "paper_2405_08578_amd", "csrc", "match.hip")


def measured_traffic():
    """HBM bytes per launch of the contraction kernel from the committed PMC
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sha = hashlib.sha256(open(MATCH_SRC, "rb").read()).hexdigest()
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("match.hip sha256") != sha:
        return None
    try:
        return float(vals["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(pair, Ls, nq_sample):
    """The FP64 oracle on the host: detect+orient+describe both full images,
    then the brute-force matcher for a sample of reference descriptors against
    all registered ones, scaled to the full query count."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    _, _, dA = oracle.features(pair.A, Ls)
    _, _, dB = oracle.features(pair.B, Ls)
    t_dd = time.perf_counter() - t0
    idx = np.random.default_rng(0).choice(len(dA), min(nq_sample, len(dA)), replace=False)
    t0 = time.perf_counter()
    oracle.match(np.ascontiguousarray(dA[idx]), dB)
    t_m = time.perf_counter() - t0
    t_pair = t_dd + t_m * len(dA) / len(idx)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / t_pair, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle: detect+describe of both {pair.A.shape[1]}x{pair.A.shape[0]} "
                       f"images ({t_dd:.2f} s) + match of {len(idx)} of {len(dA)} reference "
                       f"descriptors vs all {len(dB)} ({t_m:.2f} s), scaled to the full pair"),
            "seconds_per_pair": t_pair}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(images and match pairs would shard across GPUs with no reduction)",
              file=sys.stderr)
        sys.exit(2)

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

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        lp.detect(imgs, P, out=kps, stream=stream)
        lp.describe(imgs, kps, P, workspace=ws_d, theta=theta, desc=desc, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        lp.match([desc[0]], [desc[1]], workspace=ws_m, out=mout, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    if args.copy_probe_mb > 0:
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    dd_ms = [e[0].elapsed_time(e[1]) for e in evs]
    m_ms = [e[1].elapsed_time(e[2]) for e in evs]
    ms_per_step = 1000.0 * wall / args.steps
    pairs_per_s = 1000.0 / ms_per_step
    mpix = 2 * h * w / 1e6
    dd_avg = sum(dd_ms) / len(dd_ms)
    m_avg = sum(m_ms) / len(m_ms)
    flops = 2.0 * n_kp * n_kp * 128
    achieved = flops / (m_avg * 1e-3) / 1e12
    n_match = int((mout[0]["match"] >= 0).sum().item())

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
        "detect_describe_mpix_per_s": round(mpix / (dd_avg * 1e-3), 1),
        "detect_describe_ms": round(dd_avg, 4),
        "match_ms": round(m_avg, 4),
        "matches": n_match,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4),
                     "traffic": measured_traffic(),
                     "kernel": "matcher call (norms + FP32 MFMA contraction/top-k + rescore), "
                               f"{flops / 1e9:.1f} GFLOP per call"},
    }
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
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        for _ in range(args.steps):
            call()
        e[1].record(stream)
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1]) / args.steps
        same = (outl[0]["match"] == ref).float().mean().item()
        lowp[name] = {"match_ms": round(ms, 4),
                      "pairs_per_s": round(1000.0 / (dd_avg + ms), 2),
                      "contraction_tflops_equiv": round(flops / (ms * 1e-3) / 1e12, 1),
                      "list_agreement_with_fp32": round(same, 6)}
        if prec == 3:
            lowp[name]["queries_rematched_fp32"] = int(stats.item())
        del wsl, outl
    out["low_precision_match"] = lowp

    if not args.no_cpu_baseline:
        cb = cpu_baseline(pair, Ls, args.cpu_queries)
        out["cpu_baseline"] = {k: (round(v, 6) if isinstance(v, float) else v)
                               for k, v in cb.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
