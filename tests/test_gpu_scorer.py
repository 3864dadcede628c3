"""GPU parity of the learned scorer's kernels against the FP64 oracle
(oracle/scorer.py).

 * score: the oracle MLP on the oracle's features, with W1 and W2 rounded to
   BF16 by torch (the kernel's weight precision). The remaining differences are
   the BF16 rounding of h1 (relative 2^-9) and FP32 accumulation, so the
   tolerance per keypoint is 2^-8 sum_j |w3_j| sum_k |W2_jk| h1_k plus 1e-5 of
   the magnitudes of all three layers' terms.
 * prune: bit-exact against the oracle prune of the GPU's own scores.
 * describe_selected: bit-identical to the full describe at the listed slots.
 * gather: patches exact, scale feature to FP32 rounding, contrast exact.
 * training step: the loss, and the gradient read back from Adam's first moment
   (m = 0.1 g after one step from zero), against the oracle in FP64.
"""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from oracle import scorer as S
from gpu_util import kp_numpy, say, to_dev

pytestmark = pytest.mark.gpu


def texture(h, w, seed, n_blobs):
    rng = np.random.Generator(np.random.PCG64(seed))
    cv = synth.render_texture(0, 0, w, h, n_blobs, rng)
    return synth.to_uint8(cv.tex, rng)


def weights(seed=0, bias_scale=0.1):
    rng = np.random.default_rng(seed)
    th = synth.scorer_init(rng)
    # non-zero biases, so that every term of the forward pass is exercised
    p = S.unflatten(th)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.uniform(-bias_scale, bias_scale, p[k].shape)
    return S.flatten(p).astype(np.float32)


def bf16_weights(w32):
    """The kernel's weights: W1 and W2 rounded to BF16 (torch's RNE), rest FP32."""
    import torch
    th = w32.astype(np.float64)
    p = S.unflatten(th)
    for k in ("W1", "W2"):
        p[k] = torch.tensor(p[k], dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    return S.flatten(p)


def score_tolerance(th, X):
    p = S.unflatten(th)
    z, (a1, h1, a2, h2) = S.forward(th, X)
    aw3 = np.abs(p["w3"])
    aW2 = np.abs(p["W2"])
    T2 = (h1 @ aW2.T) @ aw3
    T1 = ((np.abs(X) @ np.abs(p["W1"]).T) @ aW2.T) @ aw3
    T3 = h2 @ aw3 + abs(p["b3"][0])
    return z, 2.0 ** -8 * T2 + 1e-5 * (T1 + T2 + T3) + 1e-6


def run_score(gpu, img, Ls, w32):
    import torch
    P = lp.Params(Ls)
    t = to_dev(img, gpu)
    kps = lp.detect([t], P)
    sc = lp.score([t], kps, P, torch.from_numpy(w32).to(gpu))
    return t, P, kps, sc


@pytest.mark.parametrize("h,w,Ls,seed", [(150, 200, [8, 16, 32], 0), (37, 29, [4, 8], 1),
                                         (96, 130, [16], 2)])
def test_score_matches_oracle(gpu, h, w, Ls, seed):
    img = texture(h, w, seed, max(4, h * w // 400))
    w32 = weights(seed)
    say("score", h, w, Ls)
    t, P, kps, sc = run_score(gpu, img, Ls, w32)
    k = kp_numpy(kps[0])
    X = S.features(img, k["x"], k["y"], k["scale"], k["contrast"], Ls)
    z, tol = score_tolerance(bf16_weights(w32), X)
    g = sc[0].cpu().numpy().astype(np.float64)
    err = np.abs(g - z)
    assert np.all(err <= tol), f"max err {err.max()}, worst ratio {(err / tol).max()}"


def test_score_config1_sampled(gpu):
    pair = synth.config_pair(1)
    Ls = [16, 32, 64, 128]
    w32 = weights(5, bias_scale=0.5)
    say("score config 1 sampled")
    t, P, kps, sc = run_score(gpu, pair.A, Ls, w32)
    k = kp_numpy(kps[0])
    idx = np.sort(np.random.default_rng(1).choice(len(k["x"]), 400, replace=False))
    X = S.features(pair.A, k["x"][idx], k["y"][idx], k["scale"][idx], k["contrast"][idx], Ls)
    z, tol = score_tolerance(bf16_weights(w32), X)
    g = sc[0].cpu().numpy().astype(np.float64)[idx]
    assert np.all(np.abs(g - z) <= tol)
    assert np.std(z) > 0.01           # scores are not degenerate


def test_prune_matches_oracle_on_gpu_scores(gpu):
    import torch
    img = texture(300, 420, 3, 300)
    Ls = [8, 16, 32, 64]
    t, P, kps, sc = run_score(gpu, img, Ls, weights(3))
    s = sc[0].cpu().numpy()
    for k in (0, 1, lp.keep_count(len(s)), len(s) - 1, len(s)):
        say("prune", len(s), k)
        got = lp.prune([sc[0]], [k])[0].cpu().numpy()
        assert np.array_equal(got, S.prune(s, k)), k


@pytest.mark.parametrize("n,levels,seed", [(1, 1, 0), (1000, 3, 1), (70001, 5, 2),
                                           (4097, 100000, 3)])
def test_prune_ties_and_signs(gpu, n, levels, seed):
    import torch
    rng = np.random.default_rng(seed)
    s = (rng.integers(0, levels, n) - levels // 2).astype(np.float32) * np.float32(0.37)
    s[rng.integers(0, n, max(1, n // 10))] = -0.0            # -0 equals +0
    ks = [0, 1, n // 2, lp.keep_count(n), n]
    ts = [torch.from_numpy(s).to(gpu) for _ in ks]
    say("prune ties", n, levels)
    out = lp.prune(ts, ks)
    for kk, o in zip(ks, out):
        assert np.array_equal(o.cpu().numpy(), S.prune(s, kk)), kk


def test_prune_many_images(gpu):
    import torch
    rng = np.random.default_rng(9)
    scores = [torch.from_numpy(rng.normal(size=int(m)).astype(np.float32)).to(gpu)
              for m in rng.integers(1, 3000, 21)]                  # two launches
    ks = [lp.keep_count(s.numel()) for s in scores]
    say("prune 21 images")
    out = lp.prune(scores, ks)
    for s, k, o in zip(scores, ks, out):
        assert np.array_equal(o.cpu().numpy(), S.prune(s.cpu().numpy(), k))


def test_describe_selected_equals_full(gpu):
    import torch
    imgs = [texture(200, 260, 4, 150), texture(123, 301, 5, 120)]
    Ls = [8, 16, 32]
    P = lp.Params(Ls)
    ts = [to_dev(i, gpu) for i in imgs]
    kps, th, de = lp.features(ts, P)
    rng = np.random.default_rng(2)
    sels = []
    for kp in kps:
        n = kp["x"].numel()
        sels.append(np.sort(rng.choice(n, n // 3, replace=False)).astype(np.int32))
    sels[1] = np.concatenate([sels[1], np.array([-1, kps[1]["x"].numel()], np.int32)])  # invalid
    say("describe selected")
    th_s, de_s = lp.describe_selected(ts, kps, P, [torch.from_numpy(s).to(gpu) for s in sels])
    for i, s in enumerate(sels):
        ok = (s >= 0) & (s < kps[i]["x"].numel())
        full_t, full_d = th[i].cpu().numpy(), de[i].cpu().numpy()
        gt, gd = th_s[i].cpu().numpy(), de_s[i].cpu().numpy()
        assert np.array_equal(gt[ok], full_t[s[ok]])
        assert np.array_equal(gd[ok], full_d[s[ok]])
        assert np.all(np.isnan(gt[~ok])) and np.all(gd[~ok] == 0)


def test_gather_matches_oracle_features(gpu):
    import torch
    img = texture(90, 110, 6, 60)
    Ls = [4, 8, 16]
    P = lp.Params(Ls)
    t = to_dev(img, gpu)
    kps = lp.detect([t], P)
    k = kp_numpy(kps[0])
    sel = np.array([0, 5, len(k["x"]) - 1, 17, 17], np.int32)
    say("gather")
    pa, ex = lp.scorer_gather([t], kps, P, [torch.from_numpy(sel).to(gpu)])
    X = S.features(img, k["x"][sel], k["y"][sel], k["scale"][sel], k["contrast"][sel], Ls)
    assert np.array_equal(pa[0].cpu().numpy().astype(np.float64) / 255.0, X[:, :256])
    e = ex[0].cpu().numpy()
    assert np.allclose(e[:, 0], X[:, 256], rtol=1e-7, atol=0)
    assert np.array_equal(e[:, 1], X[:, 257].astype(np.float32))
    pa2, ex2 = lp.scorer_gather([t], kps, P)                   # every slot
    assert pa2[0].shape[0] == len(k["x"])
    assert np.array_equal(pa2[0].cpu().numpy()[sel], pa[0].cpu().numpy())


def training_batch(gpu, n, seed, h=160, w=200):
    import torch
    img = texture(h, w, seed, h * w // 260)
    Ls = [8, 16, 32]
    P = lp.Params(Ls)
    t = to_dev(img, gpu)
    kps = lp.detect([t], P)
    k = kp_numpy(kps[0])
    rng = np.random.default_rng(seed)
    sel = rng.choice(len(k["x"]), n, replace=False).astype(np.int32)
    pa, ex = lp.scorer_gather([t], kps, P, [torch.from_numpy(sel).to(gpu)])
    X = S.features(img, k["x"][sel], k["y"][sel], k["scale"][sel], k["contrast"][sel], Ls)
    y = (rng.uniform(size=n) < 0.3).astype(np.float32)
    m = np.where(y > 0, 2.0, 1.0).astype(np.float32)
    return pa[0], ex[0], X, y, m


def test_train_step_matches_oracle(gpu):
    import torch
    pa, ex, X, y, m = training_batch(gpu, 300, 7)
    w32 = weights(8)
    th = w32.astype(np.float64)
    tr = lp.ScorerTrainer(torch.from_numpy(w32.copy()).to(gpu), 512)
    say("train step")
    tr.step(pa, ex, torch.from_numpy(y).to(gpu), torch.from_numpy(m).to(gpu), lr=1e-3)
    torch.cuda.synchronize()
    L = S.loss(th, X, y.astype(np.float64), m.astype(np.float64))
    assert abs(tr.loss.item() - L) <= 1e-4 * abs(L)
    g = S.gradient(th, X, y.astype(np.float64), m.astype(np.float64))
    g_gpu = tr.m.cpu().numpy().astype(np.float64) / 0.1
    scale = np.abs(g).max()
    assert np.allclose(g_gpu, g, rtol=1e-3, atol=1e-5 * scale)
    # Adam's first step where the gradient is well above eps: -lr g / |g|
    th1, _, _ = S.adam(th, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    big = np.abs(g) > 1e-3 * scale
    assert np.allclose(tr.weights.cpu().numpy()[big], th1[big], rtol=0, atol=2e-5)


def test_training_learns_and_is_deterministic(gpu):
    import torch
    pa, ex, X, _, _ = training_batch(gpu, 2000, 11, 300, 400)
    # a learnable target: bright patches
    y = (X[:, :256].mean(axis=1) > np.median(X[:, :256].mean(axis=1))).astype(np.float32)
    m = np.ones_like(y)
    ty, tm = torch.from_numpy(y).to(gpu), torch.from_numpy(m).to(gpu)
    runs = []
    for r in range(2):
        tr = lp.ScorerTrainer(torch.from_numpy(weights(12)).to(gpu), 2048)
        losses = []
        say("train run", r)
        for step in range(150):
            tr.step(pa, ex, ty, tm, lr=3e-3)
            losses.append(tr.loss.item())
        runs.append((tr.weights.cpu().numpy(), losses))
    assert np.array_equal(runs[0][0], runs[1][0])             # bit-identical reruns
    l = runs[0][1]
    assert l[-1] < 0.5 * l[0], (l[0], l[-1])
