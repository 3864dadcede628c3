"""Pins of the scorer oracle (oracle/scorer.py) against independent routes:
NumPy padding and slicing for the patch features, closed forms for the scale
feature and zero padding, torch FP64 autograd and central finite differences
for the MLP and its BCE gradient, torch's Adam and the closed form of Adam's
first step, and a brute-force sort for the prune."""
import math

import numpy as np
import pytest

import synth
from oracle import scorer as S


def theta0(seed=0):
    return synth.scorer_init(np.random.default_rng(seed))


def test_param_count():
    assert S.N_PARAMS == 20801 == len(theta0())


def test_features_against_padded_slices():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (37, 45), dtype=np.uint8)
    pad = np.pad(img.astype(np.float64) / 255.0, 8)
    xs = np.array([0, 44, 20, 3, 44, 7])
    ys = np.array([0, 36, 18, 36, 0, 9])
    sc = np.array([0, 1, 2, 3, 0, 2])
    ct = np.array([0.5, 0.25, 0.0, 1.0, 0.125, 0.75])
    Ls = [16, 32, 64, 128]
    X = S.features(img, xs, ys, sc, ct, Ls)
    for i in range(len(xs)):
        # patch row r, column c = image (y + r - 8, x + c - 8), i.e. padded (y + r, x + c)
        ref = pad[ys[i]:ys[i] + 16, xs[i]:xs[i] + 16].ravel()
        assert np.array_equal(X[i, :256], ref)
    assert np.allclose(X[:, 256], np.array([0, 1, 2, 3, 0, 2]) / 3.0, rtol=0, atol=1e-15)
    assert np.array_equal(X[:, 257], ct)


def test_features_zero_padding_closed_form():
    img = np.full((30, 30), 255, np.uint8)
    X = S.features(img, np.array([0, 29, 15]), np.array([0, 29, 15]), np.zeros(3, int),
                   np.zeros(3), [8])
    # corner (0,0): rows/cols -8..7 -> 8 x 8 inside; (29,29): -8..+7 clipped at 29 -> 9 x 9
    assert X[0, :256].sum() == 64 and X[1, :256].sum() == 81 and X[2, :256].sum() == 256
    assert X[0, 256] == 0.0                      # one scale: scale feature 0
    assert S.scale_feature([16, 32, 64]).tolist() == [0.0, 0.5, 1.0]


def torch_reference(theta, X, y, m):
    torch = pytest.importorskip("torch")
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o = 0
    ps = []
    for _, shape in S.SHAPES:
        n = int(np.prod(shape))
        ps.append(t[o:o + n].reshape(shape))
        o += n
    W1, b1, W2, b2, w3, b3 = ps
    Xt = torch.tensor(X, dtype=torch.float64)
    h1 = torch.relu(torch.nn.functional.linear(Xt, W1, b1))
    h2 = torch.relu(torch.nn.functional.linear(h1, W2, b2))
    z = h2 @ w3 + b3[0]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.tensor(y, dtype=torch.float64), weight=torch.tensor(m, dtype=torch.float64),
        reduction="sum") / float(np.sum(m))
    lt.backward()
    return z.detach().numpy(), float(lt.detach()), t.grad.numpy()


def batch(n=40, seed=2):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, S.N_IN))
    y = (rng.uniform(size=n) < 0.3).astype(np.float64)
    m = np.where(y > 0, 2.5, 1.0)
    return X, y, m


def test_forward_loss_gradient_match_torch():
    th = theta0(3)
    X, y, m = batch()
    z, _ = S.forward(th, X)
    zt, lt, gt = torch_reference(th, X, y, m)
    assert np.allclose(z, zt, rtol=1e-12, atol=1e-12)
    assert math.isclose(S.loss(th, X, y, m), lt, rel_tol=1e-12)
    g = S.gradient(th, X, y, m)
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_gradient_finite_differences():
    th = theta0(4)
    X, y, m = batch(25, 5)
    g = S.gradient(th, X, y, m)
    rng = np.random.default_rng(6)
    # coordinates from every parameter block
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.SHAPES])
    idx = np.concatenate([rng.integers(offs[k], offs[k + 1], 4) for k in range(len(S.SHAPES))])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (S.loss(th + e, X, y, m) - S.loss(th - e, X, y, m)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_adam_first_step_closed_form_and_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    t1, m1, v1 = S.adam(th, g, z, z, 1, 1e-3)
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # three steps against torch.optim.Adam with a fixed gradient sequence
    gs = [rng.normal(size=50) for _ in range(3)]
    p = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=2e-3)
    tt, mm, vv = th.copy(), np.zeros(50), np.zeros(50)
    for k, gk in enumerate(gs, start=1):
        p.grad = torch.tensor(gk, dtype=torch.float64)
        opt.step()
        tt, mm, vv = S.adam(tt, gk, mm, vv, k, 2e-3)
    assert np.allclose(tt, p.detach().numpy(), rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,k,levels,seed", [(1, 1, 5, 0), (10, 3, 3, 1), (100, 30, 4, 2),
                                             (257, 78, 1000, 3), (50, 0, 2, 4), (50, 50, 2, 5)])
def test_prune_brute_force(n, k, levels, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, levels, n).astype(np.float32)       # many ties
    got = S.prune(s, k)
    # brute force: rank every slot by (score desc, slot asc) with lexsort
    order = np.lexsort((np.arange(n), -s.astype(np.float64)))
    assert np.array_equal(got, np.sort(order[:k]))
    assert len(got) == k and np.all(np.diff(got) > 0)


def test_keep_count():
    assert [S.keep_count(n) for n in (0, 1, 3, 10, 11, 43396)] == [0, 1, 1, 3, 4, 13019]
