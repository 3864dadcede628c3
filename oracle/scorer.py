"""FP64 oracle of the learned keypoint scorer: candidate features, the MLP,
its BCE loss and gradients, one Adam step, and the top-k prune.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper has no learned component; the scorer is layered on its detector
(keypoints of Sec. 2.2). Readings, shared with the product by specification
only (no shared code):
  * features of a keypoint at (x, y) of an image I (258 values):
      [0, 256)  the 16 x 16 patch I(y + r - 8, x + c - 8) / 255 at index
                16 r + c, pixels outside the image 0;
      256       (log2 L_s - log2 L_min) / (log2 L_max - log2 L_min) for the
                keypoint's window size L_s (0 with one scale);
      257       the keypoint's contrast |v - window mean| / 255;
  * MLP 258 -> 64 -> 64 -> 1 with ReLU: a1 = W1 x + b1, h1 = relu(a1),
    a2 = W2 h1 + b2, h2 = relu(a2), z = w3 . h2 + b3 (the score is z);
  * loss over a batch: sum_c m_c * BCE(sigmoid(z_c), y_c) / sum_c m_c, with
    per-candidate weights m_c (class balance) and labels y_c in {0, 1};
  * Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
  * prune: the k highest scores, a larger score first and, among equal
    scores, the lower keypoint slot first; returned as ascending slots.
Pins (tests/test_oracle_scorer.py): features against hand-built patches and
the zero padding at every border; forward and gradients against torch's FP64
autograd on the CPU and against central finite differences; Adam's first
step against its closed form (-lr g / (|g| + eps)); prune against a brute-force
sort on small and tie-heavy inputs.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

N_IN = 258
N_HID = 64
PATCH = 16

# parameter layout of the flat vector (also the layout of the product's
# weight buffers): W1 [64][258], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1]
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)      # 20,801


def unflatten(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def scale_feature(Ls: Sequence[int]) -> np.ndarray:
    """Feature 256 for each scale index."""
    lg = np.log2(np.asarray(Ls, np.float64))
    if len(Ls) == 1:
        return np.zeros(1)
    return (lg - lg[0]) / (lg[-1] - lg[0])


def features(img: np.ndarray, x: np.ndarray, y: np.ndarray, scale: np.ndarray,
             contrast: np.ndarray, Ls: Sequence[int]) -> np.ndarray:
    """[n, 258] float64 features of keypoints (x, y, scale index, contrast)."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    n = len(x)
    X = np.zeros((n, N_IN))
    sf = scale_feature(Ls)
    for i in range(n):
        for r in range(PATCH):
            yy = int(y[i]) + r - PATCH // 2
            if yy < 0 or yy >= H:
                continue
            for c in range(PATCH):
                xx = int(x[i]) + c - PATCH // 2
                if 0 <= xx < W:
                    X[i, PATCH * r + c] = img[yy, xx] / 255.0
        X[i, 256] = sf[int(scale[i])]
        X[i, 257] = float(contrast[i])
    return X


def forward(theta: np.ndarray, X: np.ndarray):
    """Scores z [n] and the activations needed by backward."""
    p = unflatten(theta)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (a1, h1, a2, h2)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(theta: np.ndarray, X: np.ndarray, y: np.ndarray, m: np.ndarray) -> float:
    """Weighted mean BCE of sigmoid(z) against labels y (stable form)."""
    z, _ = forward(theta, X)
    # -[y log s + (1-y) log(1-s)] = max(z, 0) - y z + log(1 + exp(-|z|))
    per = np.maximum(z, 0.0) - y * z + np.log1p(np.exp(-np.abs(z)))
    return float(np.sum(m * per) / np.sum(m))


def gradient(theta: np.ndarray, X: np.ndarray, y: np.ndarray, m: np.ndarray) -> np.ndarray:
    """d loss / d theta (flat, same layout as theta), by the chain rule."""
    p = unflatten(theta)
    z, (a1, h1, a2, h2) = forward(theta, X)
    dz = m * (sigmoid(z) - y) / np.sum(m)          # [n]
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, p["w3"]) * (a2 > 0)           # [n, 64]
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (a1 > 0)                 # [n, 64]
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return flatten(g)


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t >= 1): returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def prune(scores: np.ndarray, k: int) -> np.ndarray:
    """Slots of the k best scores (larger first, lower slot on ties), ascending."""
    s = np.asarray(scores)
    n = len(s)
    k = max(0, min(int(k), n))
    # order: score descending, then slot ascending
    order = sorted(range(n), key=lambda i: (-float(s[i]), i))
    return np.sort(np.asarray(order[:k], dtype=np.int64))


def keep_count(n: int, num: int = 3, den: int = 10) -> int:
    """ceil(n num / den) in integers (30 % by default)."""
    return -(-int(n) * num // den)
