"""Full-size parity on the 2600x1600 pair (43,396 keypoint slots per image),
nothing sampled:
 - every slot of both images: orientation within 1e-4 rad and descriptor
   within 1e-4 relative L2 of the FP64 oracle (slots whose oracle histogram
   has a non-adjacent near-tie excepted and counted);
 - rule (i) on every query: the FP64 oracle matcher on the GPU's own
   descriptors gives the GPU's list outside the 1e-6 decision band, with d1
   and d2 within 1e-5 relative;
 - rule (ii): the oracle end to end (FP64 features, FP64 matcher) gives the
   GPU's end-to-end list outside a 1e-3 band; the count inside is reported."""
import time

import numpy as np
import pytest

import oracle
import synth
import paper_2405_08578_amd as lp
from gpu_util import (angle_diff, kp_numpy, match_margins, orientation_ambiguity, rel_l2, say,
                      to_dev)

pytestmark = pytest.mark.gpu
LS = [16, 32, 64, 128]


def test_config1_full_parity(gpu):
    import torch
    pair = synth.config_pair(1)
    say("config 1 pair, full parity: GPU features and match")
    P = lp.Params(LS)
    kps, th, de = lp.features([to_dev(pair.A, gpu), to_dev(pair.B, gpu)], P)
    r = lp.match([de[0]], [de[1]])[0]
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in r.items()}
    desc_o = []
    t0 = time.perf_counter()
    for img, kp, t, d in zip((pair.A, pair.B), kps, th, de):
        kpn = kp_numpy(kp)
        ok = oracle.detect(img, LS)
        for f in ("x", "y", "scale", "type", "value"):
            assert np.array_equal(kpn[f].astype(np.int64), ok[f].astype(np.int64)), f
        ws = oracle.subregion_sides(LS)[kpn["scale"]]
        th_o, hist = oracle.orientation(img, kpn["x"], kpn["y"], ws, return_hist=True)
        d_o = oracle.describe(img, kpn["x"], kpn["y"], ws, th_o)
        desc_o.append(d_o)
        amb = orientation_ambiguity(hist) < 1e-5
        clear = ~amb
        err = rel_l2(d.cpu().numpy().astype(np.float64), d_o)
        dth = angle_diff(t.cpu().numpy().astype(np.float64), th_o)
        assert len(err) == 43396
        assert amb.sum() <= 0.001 * len(amb), f"{amb.sum()} ambiguous orientations"
        assert np.all(dth[clear] < 1e-4), f"theta max err {dth[clear].max()}"
        assert np.all(err[clear] < 1e-4), f"desc max rel err {err[clear].max()}"
        print(f"descriptors: {clear.sum()} of {len(err)} slots checked, max rel L2 "
              f"{err[clear].max():.3g}, ambiguous {amb.sum()}", flush=True)
    t1 = time.perf_counter()
    # rule (i): every query
    A32, B32 = de[0].cpu().numpy(), de[1].cpu().numpy()
    o = oracle.match(A32.astype(np.float64), B32.astype(np.float64))
    safe = match_margins(o["d1"], o["d2"], 0.8) > 1e-6
    assert np.array_equal(g["match"][safe], o["match"][safe]), \
        f"{np.sum(g['match'][safe] != o['match'][safe])} differing lists"
    fin = np.isfinite(o["d2"])
    assert np.allclose(g["d1"], o["d1"], rtol=1e-5, atol=1e-6)
    assert np.allclose(g["d2"][fin], o["d2"][fin], rtol=1e-5, atol=1e-6)
    assert (~safe).sum() <= 20
    t2 = time.perf_counter()
    # rule (ii): oracle end to end
    oe = oracle.match(desc_o[0], desc_o[1])
    band = match_margins(oe["d1"], oe["d2"], 0.8) <= 1e-3
    assert np.array_equal(g["match"][~band], oe["match"][~band]), \
        f"{np.sum(g['match'][~band] != oe['match'][~band])} differing lists outside the band"
    # the band is reported; a loose bound keeps it from growing unnoticed
    # (2.7 % of the queries measured: non-matching queries crowd d1/d2 near 0.8)
    assert band.sum() < 0.05 * len(band)
    n_match = int((g["match"] >= 0).sum())
    assert n_match > 500
    print(f"rule (i): {len(safe)} queries, {(~safe).sum()} in the 1e-6 band; rule (ii): "
          f"{band.sum()} in the 1e-3 band; {n_match} matches; oracle describe {t1 - t0:.1f} s, "
          f"matches {t2 - t1:.1f} s + {time.perf_counter() - t2:.1f} s", flush=True)
