"""Reduced-precision matcher paths against the FP32 path and the FP64 oracle.

The split path (precision 3, FP32 as two BF16 parts) is certified: a query
whose kept candidates cannot be shown to contain the true two nearest is
re-matched by the FP32 path, so its lists must equal the FP32 path's (and pass
the oracle rule (i)) for every query away from a decision boundary. BF16
(precision 1) and FP8 (precision 2) are approximate: their quantised operands
are checked bit for bit against the oracle's BF16 / E4M3 roundings, and their
lists against the FP64 oracle (recall of the true two nearest, the recall the
quantised oracle guarantees, and the lists wherever both were recalled).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import lowp
import synth
import paper_2405_08578_amd as lp
from gpu_util import match_margins, say, to_dev
from test_gpu_match import check_rule_i, run_match

pytestmark = pytest.mark.gpu


def sets(nA, nB, seed, sigma=0.08):
    rng = np.random.Generator(np.random.PCG64(seed))
    B = synth.random_unit_rows(nB, 128, rng).astype(np.float32)
    A = synth.noisy_copies(B.astype(np.float64), rng.integers(0, nB, nA), sigma, rng).astype(np.float32)
    return A, B


@pytest.mark.parametrize("nA,nB,seed", [(1, 1, 0), (7, 3, 1), (300, 31, 2), (513, 1000, 3),
                                        (1000, 513, 4), (4099, 5003, 5)])
def test_split_equals_fp32_path(gpu, nA, nB, seed):
    A, B = sets(nA, nB, seed)
    say("split-bf16 match", nA, nB, seed)
    g32 = run_match(gpu, A, B, precision=0)
    g16 = run_match(gpu, A, B, precision=3)
    check_rule_i(A, B, g16)
    o = oracle.match(A.astype(np.float64), B.astype(np.float64))
    safe = match_margins(o["d1"], o["d2"], 0.8) > 1e-6
    assert np.array_equal(g16["match"][safe], g32["match"][safe])
    assert np.array_equal(g16["d1"][safe], g32["d1"][safe])


def test_split_forced_fallback(gpu):
    # near-duplicate candidates: scores closer than the split error bound, so
    # most queries cannot be certified and go through the FP32 path
    rng = np.random.Generator(np.random.PCG64(7))
    base = synth.random_unit_rows(1, 128, rng)
    B = base + rng.normal(0, 2e-3, (700, 128))
    B = np.abs(B) / np.linalg.norm(B, axis=1, keepdims=True)
    A = np.abs(base + rng.normal(0, 2e-3, (900, 128)))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    A, B = A.astype(np.float32), B.astype(np.float32)
    say("split forced fallback")
    import torch
    g32 = run_match(gpu, A, B, precision=0)
    stats = torch.zeros(1, dtype=torch.int32, device=gpu)
    g16 = run_match(gpu, A, B, precision=3, stats=stats)
    assert stats.item() > 100          # the fallback really ran
    check_rule_i(A, B, g16)
    o = oracle.match(A.astype(np.float64), B.astype(np.float64))
    safe = match_margins(o["d1"], o["d2"], 0.8) > 1e-6
    assert np.array_equal(g16["match"][safe], g32["match"][safe])


def test_split_mixed_batch_and_degenerate(gpu):
    import torch
    A, B = sets(600, 450, 11)
    ta, tb = torch.from_numpy(A).to(gpu), torch.from_numpy(B).to(gpu)
    empty = torch.zeros((0, 128), dtype=torch.float32, device=gpu)
    say("split batch")
    r = lp.match([ta, ta[:5], ta], [tb, tb, empty], precision=3)
    g0 = {k: v.cpu().numpy() for k, v in r[0].items()}
    check_rule_i(A, B, g0)
    g1 = {k: v.cpu().numpy() for k, v in r[1].items()}
    check_rule_i(A[:5], B, g1)
    assert np.all(r[2]["match"].cpu().numpy() == -1)


def special_rows():
    """Hand-built rows for the quantisers: ties to even in BF16 and (after
    the per-row scale) in E4M3, zeros, signs, a row whose scaled entries fall
    in the E4M3 subnormal range, and widely spread magnitudes."""
    r = np.zeros((8, 128), np.float32)
    r[0, :4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 2 ** -134]   # BF16 halves
    r[1, 0], r[1, 1:8] = 448.0, [1.0625, 1.1875, 232.0, 2 ** -10, 3 * 2 ** -10, 15 * 2 ** -10,
                                 2 ** -9]              # scale 1: E4M3 halves and subnormals
    r[2] = 0.0                                          # zero row
    r[3, ::2], r[3, 1::2] = 0.125, -0.0625              # signs
    r[4, 0], r[4, 1:] = 1.0, np.geomspace(1e-6, 0.9, 127)
    r[5, 0], r[5, 1:] = 3e-5, 1e-9                      # tiny scale
    r[6] = np.linspace(-1.0, 1.0, 128)
    r[7, :64] = 0.2
    return r


@pytest.mark.parametrize("prec", [1, 2])
def test_quantised_rows_bit_exact(gpu, prec):
    """The quantised operands of precision 1 / 2 equal the oracle's roundings
    bit for bit (values and per-row scales): random unit descriptors, the
    640x480 pair's own descriptors and hand-built rows."""
    import torch
    rng = np.random.Generator(np.random.PCG64(17))
    sets_ = [synth.random_unit_rows(3001, 128, rng).astype(np.float32), special_rows(),
             np.zeros((0, 128), np.float32)]
    pair = synth.config_pair(0)
    _, _, de = lp.features([to_dev(pair.A, gpu)], lp.Params([16, 32, 64]))
    sets_.append(de[0].cpu().numpy())
    for D in sets_:
        say("quantise rows", prec, D.shape)
        q, s = lp.quantize_lowp(torch.from_numpy(D).to(gpu), prec)
        torch.cuda.synchronize()
        if prec == 1:
            got = lowp.decode_bf16(q.cpu().numpy().view(np.uint16))
            assert np.array_equal(got, lowp.quantize_bf16(D))
        else:
            got = lowp.decode_e4m3(q.cpu().numpy())
            want, ws = lowp.quantize_fp8(D)
            assert np.array_equal(got, want)
            assert np.array_equal(s.cpu().numpy().view(np.uint32), ws.view(np.uint32))


def key_delta(nB):
    """Resolution of the quantised matchers' ranking, in squared-distance
    units (unit descriptors): a ranking key keeps the score |b|^2 + C - 2 a.b
    (C about 3, so the score is below 8) with the low ceil(log2 nB) bits of
    its FP32 mantissa given to the candidate index, an error below
    2^(bits - 23) x 8; the FP32 contraction of exact quantised products adds
    less than 1e-5. delta is twice the total: a candidate that leads another
    by more than delta in the oracle's score also leads it in the key."""
    bits = max(int(math.ceil(math.log2(max(nB, 2)))), 6)
    return 2.0 * (2.0 ** (bits - 23) * 8.0 + 1e-5)


def check_quantised_against_oracle(A, B, g, prec, floor12):
    """Parity of a quantised match against the FP64 oracle and the quantised
    oracle (oracle/lowp.py):
     - no query's d1 / d2 beats the exact nearest / second-nearest distance;
     - a query "recalls" j1 (j1 and j2) when its d1 (d1 and d2) equal the
       exact FP64 distances to FP32 rounding; every query for which the
       quantised oracle guarantees recall (oracle/lowp.recall_guaranteed)
       does recall, and the recall of (j1, j2) is at least `floor12`;
     - where (j1, j2) are recalled, the list equals the FP64 oracle's
       outside the 1e-6 decision band."""
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    o = oracle.match(A64, B64)
    D2 = (A64 ** 2).sum(1)[:, None] + (B64 ** 2).sum(1)[None, :] - 2.0 * A64 @ B64.T
    order = np.argsort(D2, axis=1, kind="stable")
    j1 = o["j1"]
    j2 = np.where(order[:, 0] == j1, order[:, 1], order[:, 0]) if B.shape[0] > 1 else \
        np.full(len(A), -1)
    tol = lambda d: 2e-6 * d + 1e-6
    fin2 = np.isfinite(o["d2"])
    assert np.all(g["d1"] >= o["d1"] - tol(o["d1"]))
    assert np.all(g["d2"][fin2] >= o["d2"][fin2] - tol(o["d2"][fin2]))
    rec1 = np.abs(g["d1"] - o["d1"]) <= tol(o["d1"])
    rec12 = rec1 & np.where(fin2, np.abs(g["d2"] - o["d2"]) <= tol(np.where(fin2, o["d2"], 0)),
                            np.isinf(g["d2"]))
    S = lowp.quantized_scores(A, B, prec)
    sure = lowp.recall_guaranteed(S, j1, j2, key_delta(B.shape[0]))
    assert np.all(rec1[sure["j1"]]), f"{np.sum(~rec1[sure['j1']])} guaranteed j1 missed"
    assert np.all(rec12[sure["j1_j2"]]), f"{np.sum(~rec12[sure['j1_j2']])} guaranteed pairs missed"
    assert rec1.mean() >= floor12 and rec12.mean() >= floor12, (rec1.mean(), rec12.mean())
    safe = rec12 & (match_margins(o["d1"], o["d2"], 0.8) > 1e-6)
    assert np.array_equal(g["match"][safe], o["match"][safe])
    print(f"precision {prec}: recall j1 {rec1.mean():.5f}, (j1, j2) {rec12.mean():.5f}; "
          f"guaranteed {sure['j1'].mean():.3f} / {sure['j1_j2'].mean():.3f}", flush=True)
    return rec1.mean(), rec12.mean()


@pytest.mark.parametrize("prec,floor12", [(1, 0.995), (2, 0.98)])
@pytest.mark.parametrize("nA,nB,seed", [(2000, 3000, 3), (4099, 5003, 5), (77, 300, 8)])
def test_quantised_against_oracle(gpu, nA, nB, seed, prec, floor12):
    A, B = sets(nA, nB, seed)
    say("quantised match", prec, nA, nB, seed)
    g = run_match(gpu, A, B, precision=prec)
    check_quantised_against_oracle(A, B, g, prec, floor12)


@pytest.mark.parametrize("prec,floor12", [(1, 0.99), (2, 0.97)])
def test_quantised_config0_descriptors(gpu, prec, floor12):
    """LP-SIFT descriptors of the 640x480 pair (neighbours much denser than
    in random sets) through the quantised matchers."""
    pair = synth.config_pair(0)
    say("quantised config 0", prec)
    _, _, de = lp.features([to_dev(pair.A, gpu), to_dev(pair.B, gpu)], lp.Params([16, 32, 64]))
    r = lp.match([de[0]], [de[1]], precision=prec)[0]
    g = {k: v.cpu().numpy() for k, v in r.items()}
    check_quantised_against_oracle(de[0].cpu().numpy(), de[1].cpu().numpy(), g, prec, floor12)


def test_config0_lists_split(gpu):
    pair = synth.config_pair(0)
    say("split config 0")
    kps, th, de = lp.features([to_dev(pair.A, gpu), to_dev(pair.B, gpu)], lp.Params([16, 32, 64]))
    r32 = lp.match([de[0]], [de[1]], precision=0)[0]
    r16 = lp.match([de[0]], [de[1]], precision=3)[0]
    A32, B32 = de[0].cpu().numpy(), de[1].cpu().numpy()
    g16 = {k: v.cpu().numpy() for k, v in r16.items()}
    check_rule_i(A32, B32, g16)
    o = oracle.match(A32.astype(np.float64), B32.astype(np.float64))
    safe = match_margins(o["d1"], o["d2"], 0.8) > 1e-6
    assert np.array_equal(g16["match"][safe], r32["match"].cpu().numpy()[safe])


def test_config1_split_equals_fp32(gpu):
    import torch
    pair = synth.config_pair(1)
    say("split config 1")
    kps, th, de = lp.features([to_dev(pair.A, gpu), to_dev(pair.B, gpu)],
                              lp.Params([16, 32, 64, 128]))
    r32 = lp.match([de[0]], [de[1]], precision=0)[0]
    stats = torch.zeros(1, dtype=torch.int32, device=gpu)
    r3 = lp.match([de[0]], [de[1]], precision=3, stats=stats)[0]
    g32 = {k: v.cpu().numpy() for k, v in r32.items()}
    g3 = {k: v.cpu().numpy() for k, v in r3.items()}
    print("re-matched in FP32:", stats.item(), flush=True)
    # both lists come from FP32 rescoring; they may differ only where the FP32
    # contraction itself cannot separate the 2nd and 3rd candidate (1e-6 band)
    diff = np.nonzero(g3["match"] != g32["match"])[0]
    if len(diff):
        marg = match_margins(g32["d1"][diff].astype(np.float64), g32["d2"][diff].astype(np.float64), 0.8)
        assert np.all(marg < 1e-5)
    assert len(diff) <= 3


@pytest.mark.parametrize("prec", [1, 2])
def test_quantised_topk(gpu, prec):
    """topk (candidates rescored in FP32 per query): 8 is the default, bit for
    bit; 2 still finds every query whose true two nearest the quantised oracle
    guarantees, and wherever it recalls both its lists equal topk 8's, since
    the rescored distances are the same FP32 values."""
    A, B = sets(2000, 3000, 3)
    say("quantised topk", prec)
    g0 = run_match(gpu, A, B, precision=prec)
    g8 = run_match(gpu, A, B, precision=prec, topk=8)
    for k in ("match", "d1", "d2"):
        assert np.array_equal(g0[k], g8[k])
    g2 = run_match(gpu, A, B, precision=prec, topk=2)
    rec1, rec12 = check_quantised_against_oracle(A, B, g2, prec, 0.5)
    r1, r12 = check_quantised_against_oracle(A, B, g8, prec, 0.5)
    assert rec12 <= r12 + 1e-12
    o = oracle.match(A.astype(np.float64), B.astype(np.float64))
    fin2 = np.isfinite(o["d2"])
    tol = lambda d: 2e-6 * d + 1e-6
    both = (np.abs(g2["d1"] - o["d1"]) <= tol(o["d1"])) & fin2 & \
        (np.abs(g2["d2"] - np.where(fin2, o["d2"], 0)) <= tol(np.where(fin2, o["d2"], 0)))
    both &= (np.abs(g8["d1"] - o["d1"]) <= tol(o["d1"])) & \
        (np.abs(g8["d2"] - np.where(fin2, o["d2"], 0)) <= tol(np.where(fin2, o["d2"], 0)))
    assert both.mean() > 0.5
    for k in ("match", "d1", "d2"):
        assert np.array_equal(g2[k][both], g8[k][both])
