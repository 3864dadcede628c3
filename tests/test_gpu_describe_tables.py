"""The disc tables that lpsift_describe builds in its workspace, read back
after a call: the orientation disc of every scale whole, and the descriptor
disc once per orientation bucket, keeping every entry that the square of
reachable subregions (|u|, |v| < 2.5 subregions after rotating the offset by
-theta, Sec. 2.3) can cover for an angle of the bucket.

Layout (16-byte entries: dx, dy as floats, the Gaussian weight times the
votes' fixed-point scale, the offset packed as two int16): per scale the
orientation disc, then 64 bucket lists of
n_desc entries each (one whole list when the disc has more than 8,192
entries); then the int32 entry counts [8 scales][64 buckets]. The geometry is
recomputed here from Eq. 3-4 as the library derives it."""
import math

import numpy as np
import pytest
import torch

import paper_2405_08578_amd as lp
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

BUCKETS = 64


def disc(r2):
    R = math.isqrt(r2)
    out = []
    for dy in range(-R, R + 1):
        hw = math.isqrt(r2 - dy * dy)
        out.extend((dx, dy) for dx in range(-hw, hw + 1))
    return out


def geometry(Ls, d=4):
    beta0 = (1.0 / d) * math.sqrt(Ls[0] / Ls[-1])
    log2e = 1.4426950408889634
    scales, entries = [], 0
    for L in Ls:
        ws = beta0 * (L / Ls[-1]) ** -0.5 * L
        half = 0.5 * (d + 1) * ws
        ro = math.floor(1.5 * ws + 0.5)
        g = {"ws": ws, "r2o": int(ro * ro), "r2d": int(math.floor(2.0 * half * half)),
             "ko": np.float32(-log2e / (2.0 * (0.5 * ws) ** 2)),
             "kd": np.float32(-log2e / (2.0 * (0.5 * d) ** 2 * ws * ws))}
        g["no"], g["nd"] = len(disc(g["r2o"])), len(disc(g["r2d"]))
        # descriptor vote scale: 362 (> the largest gradient, 255 sqrt 2) times
        # a bound on one cell's bilinear weights over the pixels, plus 1/2 per
        # vote, stays below 0.98 of 2^32
        nv = (2.0 * math.sqrt(2.0) * ws + 2.0) ** 2
        g["dscale"] = float(np.float32((0.98 * 2.0 ** 32 - 0.5 * nv) / (362.0 * (ws * ws + 4.5 * ws + 1.0))))
        g["nb"] = BUCKETS if g["nd"] <= 8192 else 1
        g["off_o"] = entries
        entries += g["no"]
        g["off_d"] = entries
        entries += g["nb"] * g["nd"]
        scales.append(g)
    return scales, entries


def entries_of(tab, off, n):
    e = tab[off:off + n]
    packed = e[:, 3].view(np.int32)
    dx = (packed << 16) >> 16
    dy = packed >> 16
    return e, dx, dy


@pytest.mark.parametrize("Ls,shape", [([16, 32, 64, 128], (129, 200)), ([16, 256], (300, 300))])
def test_tables_in_the_workspace(gpu, Ls, shape):
    say("describe tables", Ls, shape)
    rng = np.random.default_rng(0)
    img = to_dev(rng.integers(0, 256, shape, dtype=np.uint8), gpu)
    P = lp.Params(Ls)
    kps = lp.detect([img], P)
    ws = torch.zeros(lp.describe_workspace_size([img], P), dtype=torch.uint8, device=gpu)
    lp.describe([img], kps, P, workspace=ws)
    torch.cuda.synchronize()
    check_tables(ws.cpu().numpy(), Ls)


def check_tables(raw, Ls):
    scales, n_entries = geometry(Ls)
    tab = raw[:n_entries * 16].view(np.float32).reshape(-1, 4)
    coff = (n_entries * 16 + 255) // 256 * 256
    counts = raw[coff:coff + 8 * BUCKETS * 4].view(np.int32).reshape(8, BUCKETS)
    for s, g in enumerate(scales):
        # orientation disc: whole, row-major, weights exp2(r^2 k) 2^23
        e, dx, dy = entries_of(tab, g["off_o"], g["no"])
        assert list(zip(dx.tolist(), dy.tolist())) == disc(g["r2o"])
        assert np.array_equal(e[:, 0], dx.astype(np.float32))
        assert np.array_equal(e[:, 1], dy.astype(np.float32))
        w = np.exp2((dx * dx + dy * dy).astype(np.float64) * float(g["ko"])) * 2.0 ** 23
        assert np.allclose(e[:, 2], w, rtol=2e-6, atol=0)
        D = np.array(disc(g["r2d"]))
        inv = float(np.float32(1.0 / np.float32(g["ws"])))
        for b in range(g["nb"]):
            n = int(counts[s, b])
            e, dx, dy = entries_of(tab, g["off_d"] + b * g["nd"], n)
            got = list(zip(dx.tolist(), dy.tolist()))
            assert got == sorted(got, key=lambda t: (t[1], t[0])), "row-major order"
            assert len(set(got)) == n
            w = np.exp2((dx * dx + dy * dy).astype(np.float64) * float(g["kd"])) * g["dscale"]
            assert np.allclose(e[:, 2], w, rtol=3e-6, atol=0)
            if g["nb"] == 1:
                assert got == [tuple(t) for t in D.tolist()]
                continue
            have = set(got)
            # every entry a visit can accept at an angle of the bucket is listed
            for th in np.linspace(b / BUCKETS, (b + 1) / BUCKETS, 33) * 2 * math.pi:
                c, sn = math.cos(th) * inv, math.sin(th) * inv
                u = c * D[:, 0] + sn * D[:, 1]
                v = c * D[:, 1] - sn * D[:, 0]
                acc = (np.abs(u) < 2.5 + 1e-6) & (np.abs(v) < 2.5 + 1e-6)
                missing = [t for t in map(tuple, D[acc].tolist()) if t not in have]
                assert not missing, f"scale {s} bucket {b}: {missing[:5]}"
            # and nothing beyond the margin of the bucket's centre angle
            th = 2 * math.pi * (b + 0.5) / BUCKETS
            c, sn = math.cos(th) * inv, math.sin(th) * inv
            u = c * dx + sn * dy
            v = c * dy - sn * dx
            m = 2.5 + np.hypot(dx, dy) * inv * (math.pi / BUCKETS) * 1.01 + 1e-3 + 1e-5
            assert np.all((np.abs(u) < m) & (np.abs(v) < m))
            assert n < 0.75 * g["nd"]
