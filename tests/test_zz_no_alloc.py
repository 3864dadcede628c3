"""lpsift_match_noalloc, the matcher on the library's fixed per-device
scratch array, against lpsift_match on a caller workspace: the same kernels
run on both, so lists, d1, d2 and the re-match count must be bit-identical.
Two calls in a row per precision, the second on smaller sets, so the second
runs on the scratch contents the first left behind."""
import numpy as np
import pytest

import synth
import paper_2405_08578_amd as lp
from gpu_util import say


def _sets(sizes, seed):
    """Per pair (queries, candidates): unit rows and noisy copies of some of
    them, so that most queries have a clear nearest neighbour."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for nA, nB in sizes:
        B = synth.random_unit_rows(nB, 128, rng).astype(np.float32)
        if nB > 0:
            A = synth.noisy_copies(B, rng.integers(0, nB, nA), 0.03, rng).astype(np.float32)
        else:
            A = synth.random_unit_rows(nA, 128, rng).astype(np.float32)
        out.append((A, B))
    return out


CALLS = (
    # first call: three pairs, two sharing one candidate set, one with no candidates
    [(9000, 12000), (7000, 12000), (500, 0)],
    # second call: one smaller pair
    [(2100, 1500)],
)


@pytest.mark.gpu
@pytest.mark.parametrize("precision,topk", [(0, 0), (3, 0), (1, 0), (2, 0), (1, 3), (2, 2)])
def test_noalloc_equals_workspace_call(gpu, precision, topk):
    import torch
    for k, sizes in enumerate(CALLS):
        say("match_noalloc", "precision", precision, "topk", topk, "call", k, "sizes", sizes)
        sets = _sets(sizes, 7100 + 10 * precision + k)
        if k == 0 and len(sizes) > 1:
            sets[1] = (sets[1][0], sets[0][1])          # same registered set as pair 0
        dA = [torch.from_numpy(a).to(gpu) for a, _ in sets]
        dB = [torch.from_numpy(b).to(gpu) for _, b in sets]
        if k == 0 and len(sizes) > 1:
            dB[1] = dB[0]                               # shared pointer: norms computed once
        mp = lp.match_params(precision=precision, topk=topk)
        assert lp.match_workspace_size([len(a) for a, _ in sets], [len(b) for _, b in sets],
                                       mp) <= lp.NOALLOC_SCRATCH_BYTES
        out = [{"match": torch.full((len(a),), -7, dtype=torch.int32, device=gpu),
                "d1": torch.full((len(a),), -1.0, dtype=torch.float32, device=gpu),
                "d2": torch.full((len(a),), -1.0, dtype=torch.float32, device=gpu)}
               for a, _ in sets]
        st_n = torch.zeros(1, dtype=torch.int32, device=gpu)
        st_r = torch.zeros(1, dtype=torch.int32, device=gpu)
        got = lp.match_noalloc(dA, dB, precision=precision, out=out, stats=st_n, topk=topk)
        ref = lp.match(dA, dB, precision=precision, stats=st_r, topk=topk)
        torch.cuda.synchronize()
        for p, (g, r) in enumerate(zip(got, ref)):
            for f in ("match", "d1", "d2"):
                assert torch.equal(g[f], r[f]), (k, p, f)
        assert int(st_n.item()) == int(st_r.item())
        # the lists are real matches, not a shared failure
        n_pair0 = int((got[0]["match"] >= 0).sum().item())
        assert n_pair0 > 0.5 * sizes[0][0]
        if sizes[-1][1] == 0:
            assert int((got[-1]["match"] >= 0).sum().item()) == 0
