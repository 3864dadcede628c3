"""uint8 descriptors on the GPU (lpsift_quantize_u8, lpsift_match_u8) against
the integer oracle (oracle/quantized.py).

Rules: quantised bytes are bit-exact against the oracle applied to the same
FP32 descriptors; match lists, nearest indices and both distances are
bit-exact (the GPU distances are exact integers, the square roots and the
ratio test are taken in double on both sides, and the float outputs are the
same double rounded once)."""
import math

import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from oracle import quantized as Q
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def descriptor_sets(nA, nB, seed, sigma=0.08):
    """Descriptor-like FP32 sets: unit rows with the 0.2 clamp, queries noisy
    copies of half of the registered rows, the rest fresh rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = synth.random_unit_rows(max(nB, 1), 128, rng)
    b = base[:nB].astype(np.float32)
    src = rng.integers(0, max(nB, 1), nA)
    a = synth.noisy_copies(base, src, sigma, rng).astype(np.float32).reshape(nA, 128)
    fresh = rng.random(nA) < 0.5
    a[fresh] = synth.random_unit_rows(int(fresh.sum()), 128, rng).astype(np.float32)
    return np.ascontiguousarray(a), np.ascontiguousarray(b)


def check(res, qa, qb, ratio=0.8, abs_thresh=math.inf, rows=None):
    """Compare GPU lists with the oracle on queries `rows` (all by default)."""
    if rows is None:
        rows = np.arange(len(qa))
    abs_thresh = float(np.float32(abs_thresh))      # the entry point takes it as a float
    o = Q.match_u8(qa[rows], qb, ratio, abs_thresh)
    m = res["match"].cpu().numpy()[rows]
    d1 = res["d1"].cpu().numpy()[rows]
    d2 = res["d2"].cpu().numpy()[rows]
    assert np.array_equal(m, o["match"])
    assert np.array_equal(d1, o["d1"].astype(np.float32))
    assert np.array_equal(d2, o["d2"].astype(np.float32))
    # nearest index: the match when kept; otherwise recheck through d1
    kept = o["match"] >= 0
    assert np.array_equal(m[kept], o["j1"][kept])


def run(gpu, qa, qb, **kw):
    import torch
    A = torch.from_numpy(qa).to(gpu)
    B = torch.from_numpy(qb).to(gpu)
    r = lp.match_u8(A, B, **kw)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("n", [0, 1, 37, 1000, 4099])
def test_quantize_bit_exact(gpu, n):
    a, _ = descriptor_sets(n, 16, 3 + n)
    rng = np.random.default_rng(n)
    if n:
        a[0, :8] = np.array([0.0, 1 / 1024, 3 / 1024, 5 / 1024, 0.4980469, 0.5, 0.9, 1.0],
                            np.float32)       # halves to even, the clamp at 255
        a[-1] = rng.random(128).astype(np.float32) * 0.6
    say("quantize_u8", n)
    q = lp.quantize_u8(to_dev(a, gpu)).cpu().numpy()
    assert q.shape == (n, 128)
    assert np.array_equal(q, Q.quantize_u8(a))


@pytest.mark.parametrize("nA,nB,seed", [(700, 1000, 0), (513, 257, 1), (1, 256, 2), (511, 255, 3),
                                        (40, 513, 4), (1100, 2, 5), (9, 1, 6), (300, 5000, 7)])
def test_match_descriptor_sets(gpu, nA, nB, seed):
    import torch
    a, b = descriptor_sets(nA, nB, 100 + seed)
    say("match_u8 descriptors", nA, nB)
    qa = lp.quantize_u8(to_dev(a, gpu))
    qb = lp.quantize_u8(to_dev(b, gpu))
    r = lp.match_u8(qa, qb)
    torch.cuda.synchronize()
    ha, hb = qa.cpu().numpy(), qb.cpu().numpy()
    assert np.array_equal(ha, Q.quantize_u8(a)) and np.array_equal(hb, Q.quantize_u8(b))
    check(r, ha, hb)


def test_full_range_bytes_and_extremes(gpu):
    """Arbitrary bytes (the full 0..255 range) and the extreme distances:
    all-0 against all-255 rows (D = 128 * 255^2) and identical rows (D = 0)."""
    rng = np.random.default_rng(11)
    qa = rng.integers(0, 256, (600, 128), dtype=np.uint8)
    qb = rng.integers(0, 256, (900, 128), dtype=np.uint8)
    qa[0] = 0
    qb[5] = 255
    qa[1] = 255
    qb[7] = 0
    qa[2] = qb[300]
    qa[3] = 0
    qa[4] = 128
    say("match_u8 full-range bytes")
    for ratio in (0.8, math.inf, 1.0):
        check(run(gpu, qa, qb, ratio=ratio), qa, qb, ratio)
    only0 = np.zeros((3, 128), np.uint8)
    only255 = np.full((2, 128), 255, np.uint8)
    r = run(gpu, only0, only255, ratio=math.inf)
    check(r, only0, only255, math.inf)
    assert np.all(r["match"].cpu().numpy() == 0)
    assert np.all(r["d1"].cpu().numpy() == np.float32(math.sqrt(128 * 255 ** 2) / 512))


def test_ties_take_the_lowest_index(gpu):
    """Duplicated registered rows across chunk boundaries: the nearest is the
    lowest index and the second distance equals the first."""
    rng = np.random.default_rng(12)
    qb = rng.integers(0, 120, (1400, 128), dtype=np.uint8)
    for j, k in ((10, 700), (255, 256), (1000, 1300), (3, 1399)):
        qb[k] = qb[j]
    qa = np.stack([qb[j] for j in (700, 256, 1300, 1399, 10)])
    qa[4, 0] ^= 1
    say("match_u8 ties")
    r = run(gpu, qa, qb, ratio=math.inf)
    check(r, qa, qb, math.inf)
    o = Q.match_u8(qa, qb, math.inf)
    assert list(o["j1"][:4]) == [10, 255, 1000, 3]
    d1, d2 = r["d1"].cpu().numpy(), r["d2"].cpu().numpy()
    assert np.array_equal(d1[:4], d2[:4])


def test_thresholds_and_empty_sets(gpu):
    a, b = descriptor_sets(800, 1500, 21)
    qa, qb = Q.quantize_u8(a), Q.quantize_u8(b)
    say("match_u8 thresholds")
    for ratio, thr in ((0.8, 0.3), (math.inf, 0.25), (0.6, math.inf), (2.0, 1e-3)):
        check(run(gpu, qa, qb, ratio=ratio, abs_thresh=thr), qa, qb, ratio, thr)
    r = run(gpu, qa, qb[:0])
    assert np.all(r["match"].cpu().numpy() == -1)
    assert np.all(np.isinf(r["d1"].cpu().numpy())) and np.all(np.isinf(r["d2"].cpu().numpy()))
    r = run(gpu, qa[:0], qb)
    assert r["match"].numel() == 0


def test_repeat_call_reuses_workspace(gpu):
    """Two calls in a row on one workspace, the second smaller: every output is
    rewritten (no state survives a call)."""
    import torch
    a, b = descriptor_sets(2000, 3000, 31)
    qa, qb = Q.quantize_u8(a), Q.quantize_u8(b)
    A, B = torch.from_numpy(qa).to(gpu), torch.from_numpy(qb).to(gpu)
    ws = torch.empty(lp.match_u8_workspace_size(2000, 3000), dtype=torch.uint8, device=gpu)
    say("match_u8 repeat")
    lp.match_u8(A, B, workspace=ws)
    r = lp.match_u8(A[:700], B[:900], workspace=ws)
    torch.cuda.synchronize()
    check(r, qa[:700], qb[:900])


def test_full_size_sampled(gpu):
    """43396 x 43396 descriptors (the keypoint slots of a 2600 x 1600 image at
    L = 16, 32, 64, 128), the launch configuration the benchmark times; about 90
    sampled queries, among them both sides of several 512-query block edges and
    the last block, against the oracle."""
    import torch
    n = 43396
    a, b = descriptor_sets(n, n, 41)
    say("match_u8 full size", n)
    qa = lp.quantize_u8(to_dev(a, gpu))
    qb = lp.quantize_u8(to_dev(b, gpu))
    r = lp.match_u8(qa, qb)
    torch.cuda.synchronize()
    ha, hb = qa.cpu().numpy(), qb.cpu().numpy()
    rng = np.random.default_rng(5)
    rows = np.unique(np.r_[rng.integers(0, n, 80), [0, 511, 512, 1023, 1024, n - 1, n - 2,
                                                     n - 512, 43007, 43008]])
    check(r, ha, hb, rows=rows)
