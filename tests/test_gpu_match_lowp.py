"""Reduced-precision matcher paths against the FP32 path and the FP64 oracle.

The split path (precision 3, FP32 as two BF16 parts) is certified: a query
whose kept candidates cannot be shown to contain the true two nearest is
re-matched by the FP32 path, so its lists must equal the FP32 path's (and pass
the oracle rule (i)) for every query away from a decision boundary. BF16
(precision 1) and FP8 (precision 2) are approximate: they are checked for
recall of the FP32 nearest neighbour and for exact distances whenever the
nearest neighbour was found.
"""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("nA,nB,seed", [(2000, 3000, 3), (4099, 5003, 5)])
def test_quantised_recall(gpu, nA, nB, seed, prec):
    A, B = sets(nA, nB, seed)
    say("quantised match", prec, nA, nB, seed)
    g32 = run_match(gpu, A, B, precision=0)
    g8 = run_match(gpu, A, B, precision=prec)
    o = oracle.match(A.astype(np.float64), B.astype(np.float64))
    j1_same = g8["match"] == g32["match"]
    assert j1_same.mean() > 0.97
    # where the same nearest neighbour was found, its distance is the exact FP32 one
    both = (g8["match"] >= 0) & j1_same
    assert np.array_equal(g8["d1"][both], g32["d1"][both])


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
