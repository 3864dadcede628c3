"""Many pairs in one lpsift_match call.

The FP32 and split paths run up to 36 pairs per launch and compute the norms
of a registered set shared by several pairs once; every pair's lists must be
bit-identical to the same pair matched alone (the per-pair arithmetic does not
depend on the batch), and the split path's re-match count must be the sum of
the per-pair counts. One pair per call is itself checked against the oracle in
test_gpu_match.py; here one pair of the batch is checked again (rule (i)).
"""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from gpu_util import say
from test_gpu_match import check_rule_i

pytestmark = pytest.mark.gpu


def descriptor_sets(sizes, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    base = synth.random_unit_rows(max(sizes) + 1, 128, rng)
    out = []
    for n in sizes:
        src = rng.integers(0, len(base), n)
        out.append(synth.noisy_copies(base, src, 0.08, rng).astype(np.float32).reshape(n, 128))
    return out


def all_pairs(n):
    return [(i, j) for i in range(n) for j in range(n) if i != j]


def host(r):
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("prec", [0, 3, 1, 2])
def test_batch_equals_pairs_alone(gpu, prec):
    import torch
    # 42 ordered pairs: launches of 36 and 6 pairs (the counters of every job
    # of a launch are cleared and summed, which the re-match count checks)
    sizes = [700, 450, 1000, 37, 0, 260, 333]
    sets = [torch.from_numpy(s).to(gpu) for s in descriptor_sets(sizes, 40 + prec)]
    pairs = all_pairs(len(sets))
    say("batched match", prec, len(pairs), "pairs")
    st_all = torch.zeros(1, dtype=torch.int32, device=gpu)
    res = lp.match([sets[i] for i, _ in pairs], [sets[j] for _, j in pairs], precision=prec,
                   stats=st_all)
    total = 0
    for (i, j), r in zip(pairs, res):
        st = torch.zeros(1, dtype=torch.int32, device=gpu)
        alone = lp.match([sets[i]], [sets[j]], precision=prec, stats=st)[0]
        a, b = host(r), host(alone)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, j, k)
        total += st.item()
        if sizes[j] == 0:
            assert np.all(a["match"] == -1) and np.all(np.isinf(a["d1"]))
    assert st_all.item() == total
    if prec == 0:
        i, j = pairs[1]
        check_rule_i(sets[i].cpu().numpy(), sets[j].cpu().numpy(), host(res[1]))


@pytest.mark.parametrize("chunks", [1, 5, 16])
def test_batch_shared_sets_chunks(gpu, chunks):
    import torch
    sets = [torch.from_numpy(s).to(gpu) for s in descriptor_sets([900, 1300, 513], 77)]
    # the same registered set in several pairs, and a repeated pair
    pairs = [(0, 1), (2, 1), (1, 0), (2, 0), (0, 1), (1, 2)]
    say("batched match, shared sets, chunks", chunks)
    res = lp.match([sets[i] for i, _ in pairs], [sets[j] for _, j in pairs], b_chunks=chunks)
    for (i, j), r in zip(pairs, res):
        alone = lp.match([sets[i]], [sets[j]], b_chunks=chunks)[0]
        a, b = host(r), host(alone)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, j, k)
    check_rule_i(sets[2].cpu().numpy(), sets[1].cpu().numpy(), host(res[1]))


@pytest.mark.parametrize("precision", [0, 3])
def test_wave_counts_give_identical_lists(gpu, precision):
    """The FP32 contraction's workgroup shape (2, 4 or 8 wavefronts of 64
    queries) changes only the work split: lists, d1 and d2 equal bit for bit
    (the split path's FP32 re-match uses the same shape)."""
    import torch
    sets = [torch.from_numpy(s).to(gpu) for s in descriptor_sets([900, 1300, 513, 77], 91)]
    pairs = [(0, 1), (2, 1), (3, 0), (1, 3)]
    A = [sets[i] for i, _ in pairs]
    B = [sets[j] for _, j in pairs]
    for chunks in (0, 3):
        say("batched match, wave counts", precision, chunks)
        ref = [host(r) for r in lp.match(A, B, precision=precision, b_chunks=chunks, qblock_waves=4)]
        for w in (2, 8):
            got = [host(r) for r in lp.match(A, B, precision=precision, b_chunks=chunks,
                                             qblock_waves=w)]
            for a, b in zip(ref, got):
                for k in a:
                    assert np.array_equal(a[k], b[k]), (w, chunks, k)
    check_rule_i(sets[2].cpu().numpy(), sets[1].cpu().numpy(), ref[1])
