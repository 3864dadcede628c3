"""The matrix-core probes run, give identical checksums on repeated calls
(the work is deterministic) and report a positive rate for every precision."""
import math

import pytest

import paper_2405_08578_amd as lp
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["fp32", "bf16", "fp8", "int8"])
def test_probe_runs_and_is_deterministic(gpu, kind):
    import torch
    lib = lp.load()
    out = [torch.empty(int(lib.lpsift_probe_out_size()), dtype=torch.float32, device=gpu)
           for _ in range(2)]
    say("mfma probe", kind)
    for o in out:
        assert lib.lpsift_probe(lp.PROBES[kind], 16, o.data_ptr(), None) == lp.LPSIFT_OK
    torch.cuda.synchronize()
    assert torch.equal(out[0], out[1])
    assert torch.isfinite(out[0]).all() and (out[0] != 0).any()
    rate = lp.mfma_probe(kind, iters=256, reps=1, device=gpu)
    assert math.isfinite(rate) and rate > 1.0
