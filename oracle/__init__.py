"""FP64 CPU oracle of the LP-SIFT hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline import this package; the product library never does, and the oracle
never imports the product. The arithmetic lives in ``lpsift_oracle.c`` (plain
C, double precision), ``ransac.py``, ``scorer.py``, ``quantized.py``,
``multi_orient.py`` and ``warp.py`` (NumPy, double precision); this module
only marshals arrays.

Pins (what each function is checked against, in tests/test_oracle_*.py):
  detect       brute force on tiny images, Eq. 1 in exact rational arithmetic,
               closed-form images, keypoint-count and nesting invariants
  orientation  closed-form gradient ramps (bin centre, bin midpoint), the
               90-degree rotation equivariance, gain invariance
  describe     separable closed form of a constant-gradient patch, direction
               binning of a ramp, rotation and gain invariance, unit norm
  match        SciPy k-d tree / cdist cross-check, hand-built exact cases
  ransac       exact correspondences (DLT recovers H), known outlier sets
  quantized    uint8 quantisation closed forms, integer distances vs cdist,
               the (4, 5) ratio case, duplicate rows
  multi_orient secondary-peak rule on closed-form histograms (threshold,
               strictness, wrap, order, truncation, parabola), an image with
               orientations exactly {0, 90} degrees, rot90 equivariance
  warp         identity / integer translations reproduce the image, a linear
               ramp under affine and projective maps (closed form at the
               preimage), the feathered mean of two constant images,
               coverage counts, canvas bounds of known corners
  scorer       padded-slice patches, torch FP64 autograd and finite
               differences for the MLP gradient, Adam's closed-form first
               step and torch's Adam, brute-force sort for the prune
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpsift_oracle.c")
_LIB = os.path.join(_HERE, "liblpsift_oracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP on the outer loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_num_keypoints.restype = ctypes.c_int64
    lib.oracle_num_keypoints.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p]
    lib.oracle_detect.restype = None
    lib.oracle_detect.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, _f64p]
    lib.oracle_subregion_side.restype = ctypes.c_double
    lib.oracle_subregion_side.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
    lib.oracle_default_beta0.restype = ctypes.c_double
    lib.oracle_default_beta0.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_orientation.restype = None
    lib.oracle_orientation.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int64, _i32p, _i32p, _f64p, _f64p,
                                       ctypes.c_void_p]
    lib.oracle_describe.restype = None
    lib.oracle_describe.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int64, _i32p, _i32p, _f64p, _f64p,
                                    ctypes.c_int32, _f64p]
    lib.oracle_match.restype = None
    lib.oracle_match.argtypes = [_f64p, ctypes.c_int64, _f64p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, _i32p, _f64p, _f64p, _i32p]
    lib.oracle_gradient_at.restype = ctypes.c_int
    lib.oracle_gradient_at.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def _img(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim != 2:
        raise ValueError("image must be 2-D uint8")
    return img


def num_keypoints(h: int, w: int, Ls: Sequence[int]) -> int:
    Ls = np.ascontiguousarray(Ls, dtype=np.int32)
    return int(_load().oracle_num_keypoints(h, w, len(Ls), Ls))


def detect(img: np.ndarray, Ls: Sequence[int]) -> Dict[str, np.ndarray]:
    """Window maxima and minima for every L (Sec. 2.2, Eq. 2)."""
    img = _img(img)
    h, w = img.shape
    Ls = np.ascontiguousarray(Ls, dtype=np.int32)
    n = num_keypoints(h, w, Ls)
    out = {k: np.empty(n, np.int32) for k in ("x", "y", "scale", "type", "value")}
    out["contrast"] = np.empty(n, np.float64)
    _load().oracle_detect(img, h, w, w, len(Ls), Ls, out["x"], out["y"], out["scale"],
                          out["type"], out["value"], out["contrast"])
    return out


def default_beta0(Ls: Sequence[int], d: int = 4) -> float:
    return float(_load().oracle_default_beta0(d, int(min(Ls)), int(max(Ls))))


def subregion_sides(Ls: Sequence[int], d: int = 4, beta0: Optional[float] = None) -> np.ndarray:
    """w_s for each scale (Eq. 3)."""
    b0 = default_beta0(Ls, d) if beta0 is None or beta0 <= 0 else beta0
    return np.array([_load().oracle_subregion_side(int(L), int(max(Ls)), b0) for L in Ls])


def orientation(img: np.ndarray, x: np.ndarray, y: np.ndarray, ws: np.ndarray,
                return_hist: bool = False):
    img = _img(img)
    h, w = img.shape
    x = np.ascontiguousarray(x, np.int32)
    y = np.ascontiguousarray(y, np.int32)
    ws = np.ascontiguousarray(np.broadcast_to(ws, x.shape), np.float64)
    th = np.empty(len(x), np.float64)
    hist = np.empty((len(x), 36), np.float64) if return_hist else None
    _load().oracle_orientation(img, h, w, w, len(x), x, y, ws, th,
                               hist.ctypes.data if return_hist else None)
    return (th, hist) if return_hist else th


def describe(img: np.ndarray, x: np.ndarray, y: np.ndarray, ws: np.ndarray,
             theta0: np.ndarray, d: int = 4) -> np.ndarray:
    img = _img(img)
    h, w = img.shape
    x = np.ascontiguousarray(x, np.int32)
    y = np.ascontiguousarray(y, np.int32)
    ws = np.ascontiguousarray(np.broadcast_to(ws, x.shape), np.float64)
    theta0 = np.ascontiguousarray(np.broadcast_to(theta0, x.shape), np.float64)
    out = np.empty((len(x), d * d * 8), np.float64)
    _load().oracle_describe(img, h, w, w, len(x), x, y, ws, theta0, d, out)
    return out


def match(A: np.ndarray, B: np.ndarray, ratio: float = 0.8,
          abs_thresh: float = math.inf) -> Dict[str, np.ndarray]:
    """Nearest neighbour of every row of A among the rows of B (Eq. 6) with
    the ratio test."""
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    if A.ndim != 2 or B.ndim != 2 or (len(B) and A.shape[1] != B.shape[1]):
        raise ValueError("descriptor arrays must be [n, dim] with equal dim")
    nA = len(A)
    out = {"j1": np.empty(nA, np.int32), "d1": np.empty(nA, np.float64),
           "d2": np.empty(nA, np.float64), "match": np.empty(nA, np.int32)}
    if nA == 0:
        return out
    if len(B) == 0:
        B = np.zeros((0, A.shape[1]), np.float64)
    _load().oracle_match(A, nA, B, len(B), A.shape[1], float(ratio), float(abs_thresh),
                         out["j1"], out["d1"], out["d2"], out["match"])
    return out


def gradient_at(img: np.ndarray, r: int, c: int):
    img = _img(img)
    h, w = img.shape
    m, a = ctypes.c_double(), ctypes.c_double()
    if _load().oracle_gradient_at(img, h, w, w, r, c, ctypes.byref(m), ctypes.byref(a)) != 0:
        raise ValueError("pixel has no central differences")
    return m.value, a.value


def features(img: np.ndarray, Ls: Sequence[int], d: int = 4,
             beta0: Optional[float] = None, return_hist: bool = False):
    """Detect, orient and describe one image; returns (kp, theta0, desc[, hist])."""
    kp = detect(img, Ls)
    ws_scale = subregion_sides(Ls, d, beta0)
    ws = ws_scale[kp["scale"]]
    r = orientation(img, kp["x"], kp["y"], ws, return_hist=return_hist)
    th = r[0] if return_hist else r
    desc = describe(img, kp["x"], kp["y"], ws, th, d)
    return (kp, th, desc, r[1]) if return_hist else (kp, th, desc)
