"""All-pairs matching of a shuffled tile set (detect + describe of every tile,
then every pair i < j), eagerly and as a captured HIP graph.

Graph replays must reproduce the eager step bit for bit (every kernel of the
path is deterministic): each replay runs after its outputs were overwritten and
after unrelated eager work, and is checked on its own. The eager step itself is
checked against the oracle on one tile (keypoints bit-exact, a descriptor
sample within 1e-4) and on one pair (match rule (i)), at a small tile size and
at the full 2600x1600 - 2800x1800 tile size on sampled outputs.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2405_08578_amd as lp
from paper_2405_08578_amd.allpairs import AllPairs
from gpu_util import (assert_keypoints_equal, kp_numpy, orientation_ambiguity, oracle_features_at,
                      rel_l2, say, to_dev)
from test_gpu_match import check_rule_i

pytestmark = pytest.mark.gpu


def small_tiles(seed=5):
    return synth.make_tiles(world_w=1400, world_h=900, tile_w=(520, 560), tile_h=(320, 360),
                            seed=seed)


def snapshot(ap):
    out = {"kp": [kp_numpy(k) for k in ap.kps],
           "theta": [t.cpu().numpy() for t in ap.theta],
           "desc": [d.cpu().numpy() for d in ap.desc],
           "lists": [{k: v.cpu().numpy() for k, v in o.items()} for o in ap.out],
           "stats": int(ap.stats.item())}
    return out


def scramble(ap):
    for k in ap.kps:
        for v in k.values():
            v.fill_(7)
    for t in ap.theta:
        t.fill_(float("nan"))
    for d in ap.desc:
        d.fill_(float("nan"))
    for o in ap.out:
        o["match"].fill_(-7)
        o["d1"].fill_(-1.0)
        o["d2"].fill_(-1.0)
    ap.stats.fill_(12345)


def assert_same(a, b):
    for f in ("kp", "theta", "desc", "lists"):
        for x, y in zip(a[f], b[f]):
            if isinstance(x, dict):
                for k in x:
                    assert np.array_equal(x[k], y[k]), (f, k)
            else:
                assert np.array_equal(x, y, equal_nan=False), f
    assert a["stats"] == b["stats"]


def check_oracle(tiles, ap, Ls, tile_k, pair_k, n_desc=None, n_query=None, seed=0):
    rng = np.random.default_rng(seed)
    img = tiles.images[tile_k]
    kpn = kp_numpy(ap.kps[tile_k])
    assert_keypoints_equal(kpn, oracle.detect(img, Ls))
    n = len(kpn["x"])
    idx = None if n_desc is None else np.sort(rng.choice(n, n_desc, replace=False))
    th_o, d_o, hist = oracle_features_at(img, kpn, Ls, idx)
    de = ap.desc[tile_k].cpu().numpy()
    de = de if idx is None else de[idx]
    ok = orientation_ambiguity(hist) >= 1e-5
    assert ok.mean() > 0.99
    assert np.all(rel_l2(de.astype(np.float64), d_o)[ok] < 1e-4)
    i, j = ap.pairs[pair_k]
    A = ap.desc[i].cpu().numpy()
    B = ap.desc[j].cpu().numpy()
    g = {k: v.cpu().numpy() for k, v in ap.out[pair_k].items()}
    if n_query is not None:
        q = np.sort(rng.choice(len(A), n_query, replace=False))
        A = A[q]
        g = {k: v[q] for k, v in g.items()}
    check_rule_i(A, B, g)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_allpairs_graph_replays(gpu, prec):
    import torch
    tiles = small_tiles()
    Ls = [16, 32, 64]
    imgs = [to_dev(t, gpu) for t in tiles.images]
    ap = AllPairs(imgs, lp.Params(Ls), precision=prec)
    assert len(ap.pairs) == 36
    say("all pairs eager", prec)
    ap.run()
    torch.cuda.synchronize()
    ref = snapshot(ap)
    if prec in (0, 3):            # the exact paths; BF16 / FP8 are approximate
        check_oracle(tiles, ap, Ls, tile_k=4, pair_k=10)
    say("all pairs capture", prec)
    ap.capture()
    torch.cuda.synchronize()
    other = torch.from_numpy(synth.random_unit_rows(300, 128, np.random.default_rng(1))
                             .astype(np.float32)).to(gpu)
    for r in range(3):
        scramble(ap)
        lp.match([other], [torch.flip(other, [0])])               # unrelated eager work
        torch.cuda.synchronize()
        say("all pairs replay", prec, r)
        ap.replay()
        torch.cuda.synchronize()
        assert_same(snapshot(ap), ref)


def test_allpairs_tune_small(gpu, tmp_path):
    tiles = small_tiles(6)
    imgs = [to_dev(t, gpu) for t in tiles.images[:4]]
    ap = AllPairs(imgs, lp.Params([16, 32, 64]))
    ap.run()
    A = [ap.desc[i] for i, _ in ap.pairs]
    B = [ap.desc[j] for _, j in ap.pairs]
    cache = str(tmp_path / "tune.json")
    say("match tune")
    r = lp.match_tune(A, B, candidates=(1, 2, 4), waves=(2, 4, 8), reps=1, cache=cache)
    assert r["b_chunks"] in (1, 2, 4) and r["qblock_waves"] in (2, 4, 8) and not r["cached"]
    assert len(r["ms"]) == 3 and all(len(row) == 3 for row in r["ms"])
    assert all(m > 0 for row in r["ms"] for m in row)
    best = r["ms"][r["waves"].index(r["qblock_waves"])][r["candidates"].index(r["b_chunks"])]
    assert best == min(m for row in r["ms"] for m in row)
    r2 = lp.match_tune(A, B, candidates=(1, 2, 4), waves=(2, 4, 8), reps=1, cache=cache)
    assert r2["cached"] and (r2["b_chunks"], r2["qblock_waves"]) == (r["b_chunks"], r["qblock_waves"])
    # the tuned split gives lists that pass the oracle rule
    out = lp.match(A, B, b_chunks=r["b_chunks"], qblock_waves=r["qblock_waves"])
    i, j = ap.pairs[0]
    check_rule_i(ap.desc[i].cpu().numpy(), ap.desc[j].cpu().numpy(),
                 {k: v.cpu().numpy() for k, v in out[0].items()})


def test_allpairs_full_tiles_sampled(gpu):
    import torch
    tiles = synth.make_tiles()
    Ls = [16, 32, 64, 128]
    imgs = [to_dev(t, gpu) for t in tiles.images]
    ap = AllPairs(imgs, lp.Params(Ls))
    say("all pairs full tiles, graph")
    ap.capture()
    ap.replay()
    torch.cuda.synchronize()
    check_oracle(tiles, ap, Ls, tile_k=2, pair_k=17, n_desc=400, n_query=512, seed=3)
    # overlapping tiles do match
    assert max(int((o["match"] >= 0).sum()) for o in ap.out) > 1000


def test_allpairs_u8_graph_replays(gpu):
    """The uint8 variant of the step (quantise every set, exact integer match
    of every pair): lists bit-exact against the integer oracle on the step's
    own uint8 descriptors, and graph replays bit-identical to the eager step."""
    import torch
    from oracle import quantized as Q
    tiles = small_tiles(7)
    Ls = [16, 32, 64]
    imgs = [to_dev(t, gpu) for t in tiles.images]
    ap = AllPairs(imgs, lp.Params(Ls), u8=True)
    say("all pairs u8 eager")
    ap.run()
    torch.cuda.synchronize()
    ref = snapshot(ap)
    q = [t.cpu().numpy() for t in ap.q]
    for k in (0, 5):
        assert np.array_equal(q[k], Q.quantize_u8(ref["desc"][k]))
    for pk in (0, 17, 35):
        i, j = ap.pairs[pk]
        o = Q.match_u8(q[i], q[j], 0.8)
        g = ref["lists"][pk]
        assert np.array_equal(g["match"], o["match"])
        assert np.array_equal(g["d1"], o["d1"].astype(np.float32))
        assert np.array_equal(g["d2"], o["d2"].astype(np.float32))
    say("all pairs u8 capture")
    ap.capture()
    torch.cuda.synchronize()
    for r in range(3):
        scramble(ap)
        for t in ap.q:
            t.fill_(3)
        torch.cuda.synchronize()
        say("all pairs u8 replay", r)
        ap.replay()
        torch.cuda.synchronize()
        got = snapshot(ap)
        got["stats"] = ref["stats"]          # the uint8 step does not touch the counter
        assert_same(got, ref)
