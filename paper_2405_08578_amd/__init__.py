"""LP-SIFT on AMD Instinct MI355X: Python binding of liblpsift.

Argument marshalling only. Every step of the path (detection, orientation,
description, matching) runs in the HIP kernels of liblpsift.so; PyTorch
supplies device memory and the current stream. There is no CPU fallback: if the
library is not built, every call raises.

    import paper_2405_08578_amd as lp
    P = lp.Params([16, 32, 64, 128])
    kp = lp.detect([img_a, img_b], P)              # uint8 [H, W] CUDA tensors
    theta, desc = lp.describe([img_a, img_b], kp, P)
    m = lp.match([desc[0]], [desc[1]], ratio=0.8)[0]
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblpsift.so")

LPSIFT_OK = 0
LPSIFT_EINVAL = -1
LPSIFT_ECAPACITY = -2
LPSIFT_EHIP = -3
LPSIFT_EUNSUPPORTED = -4
MAX_SCALES = 8
DESC_DIM = 128

c_i32, c_i64, c_f32, c_f64, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                    ctypes.c_double, ctypes.c_void_p)


class lpsift_params(ctypes.Structure):
    _fields_ = [("n_scales", c_i32), ("L", c_i32 * MAX_SCALES), ("d", c_i32), ("beta0", c_f32)]


class lpsift_image(ctypes.Structure):
    _fields_ = [("data", c_vp), ("height", c_i32), ("width", c_i32), ("pitch", c_i64)]


class lpsift_keypoints(ctypes.Structure):
    _fields_ = [("x", c_vp), ("y", c_vp), ("scale", c_vp), ("type", c_vp), ("value", c_vp),
                ("contrast", c_vp), ("capacity", c_i64)]


class lpsift_ransac_params(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("tries", ctypes.c_int32), ("thresh", ctypes.c_double),
                ("uniforms", ctypes.c_void_p)]


class lpsift_match_params(ctypes.Structure):
    _fields_ = [("ratio", c_f64), ("abs_thresh", c_f32), ("precision", c_i32),
                ("b_chunks", c_i32), ("qblock_waves", c_i32), ("topk", c_i32), ("stats", c_vp)]


EXPORTS = ("lpsift_version", "lpsift_status_string", "lpsift_num_keypoints", "lpsift_detect",
           "lpsift_describe_workspace_size", "lpsift_describe", "lpsift_match_workspace_size",
           "lpsift_match", "lpsift_match_tune", "lpsift_timing_enable", "lpsift_timing_read",
           "lpsift_describe_selected", "lpsift_score", "lpsift_prune", "lpsift_scorer_gather",
           "lpsift_scorer_train_workspace_size", "lpsift_scorer_train_step", "lpsift_ransac_host",
           "lpsift_ransac_workspace_size", "lpsift_ransac", "lpsift_quantize_u8",
           "lpsift_match_u8_workspace_size", "lpsift_match_u8",
           "lpsift_describe_multi_workspace_size", "lpsift_describe_multi",
           "lpsift_warp_blend", "lpsift_probe_out_size", "lpsift_probe_ops", "lpsift_probe",
           "lpsift_quantize_lowp", "lpsift_match_noalloc", "lpsift_refine_host")

_lib = None


class LpsiftError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {status} ({status_string(status)})")


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblpsift.so and declare its C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblpsift.so is not built ({path}); run "
                           "`python -m paper_2405_08578_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.lpsift_version.restype = ctypes.c_int
    lib.lpsift_version.argtypes = []
    lib.lpsift_status_string.restype = ctypes.c_char_p
    lib.lpsift_status_string.argtypes = [ctypes.c_int]
    lib.lpsift_num_keypoints.restype = c_i64
    lib.lpsift_num_keypoints.argtypes = [c_i32, c_i32, P(lpsift_params)]
    lib.lpsift_detect.restype = ctypes.c_int
    lib.lpsift_detect.argtypes = [P(lpsift_image), c_i32, P(lpsift_params), P(lpsift_keypoints), c_vp]
    lib.lpsift_describe_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_describe_workspace_size.argtypes = [P(lpsift_image), c_i32, P(lpsift_params)]
    lib.lpsift_describe.restype = ctypes.c_int
    lib.lpsift_describe.argtypes = [P(lpsift_image), c_i32, P(lpsift_keypoints), P(lpsift_params),
                                    c_vp, ctypes.c_size_t, P(c_vp), P(c_vp), c_vp]
    lib.lpsift_match_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_match_workspace_size.argtypes = [P(c_i64), P(c_i64), c_i32, P(lpsift_match_params)]
    lib.lpsift_match.restype = ctypes.c_int
    lib.lpsift_match.argtypes = [P(c_vp), P(c_i64), P(c_vp), P(c_i64), c_i32,
                                 P(lpsift_match_params), c_vp, ctypes.c_size_t, P(c_vp), P(c_vp),
                                 P(c_vp), c_vp]
    lib.lpsift_match_noalloc.restype = ctypes.c_int
    lib.lpsift_match_noalloc.argtypes = [P(c_vp), P(c_i64), P(c_vp), P(c_i64), c_i32,
                                         P(lpsift_match_params), P(c_vp), P(c_vp), P(c_vp), c_vp]
    lib.lpsift_match_tune.restype = ctypes.c_int
    lib.lpsift_match_tune.argtypes = [P(c_vp), P(c_i64), P(c_vp), P(c_i64), c_i32,
                                      P(lpsift_match_params), P(c_i32), c_i32, P(c_i32), c_i32,
                                      c_i32, c_vp, ctypes.c_size_t, P(c_vp), P(c_vp), P(c_vp),
                                      P(c_f32), P(c_i32), P(c_i32), c_vp]
    lib.lpsift_timing_enable.restype = ctypes.c_int
    lib.lpsift_timing_enable.argtypes = [c_i32]
    lib.lpsift_timing_read.restype = ctypes.c_int
    lib.lpsift_timing_read.argtypes = [c_i32, P(c_f64), P(c_i64)]
    lib.lpsift_describe_selected.restype = ctypes.c_int
    lib.lpsift_describe_selected.argtypes = [P(lpsift_image), c_i32, P(lpsift_keypoints),
                                             P(lpsift_params), P(c_vp), P(c_i64), c_vp,
                                             ctypes.c_size_t, P(c_vp), P(c_vp), c_vp]
    lib.lpsift_score.restype = ctypes.c_int
    lib.lpsift_score.argtypes = [P(lpsift_image), c_i32, P(lpsift_keypoints), P(lpsift_params),
                                 c_vp, P(c_vp), c_vp]
    lib.lpsift_prune.restype = ctypes.c_int
    lib.lpsift_prune.argtypes = [P(c_vp), P(c_i64), P(c_i64), c_i32, P(c_vp), c_vp]
    lib.lpsift_scorer_gather.restype = ctypes.c_int
    lib.lpsift_scorer_gather.argtypes = [P(lpsift_image), c_i32, P(lpsift_keypoints),
                                         P(lpsift_params), P(c_vp), P(c_i64), P(c_vp), P(c_vp),
                                         c_vp]
    lib.lpsift_scorer_train_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_scorer_train_workspace_size.argtypes = [c_i64]
    lib.lpsift_scorer_train_step.restype = ctypes.c_int
    lib.lpsift_scorer_train_step.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp,
                                             c_i64, c_f32, c_vp, ctypes.c_size_t, c_vp, c_vp]
    lib.lpsift_ransac_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_ransac_workspace_size.argtypes = [P(c_i64), c_i32, c_i32]
    lib.lpsift_ransac.restype = ctypes.c_int
    lib.lpsift_ransac.argtypes = [P(lpsift_keypoints), P(lpsift_keypoints), P(c_vp), P(c_vp), P(c_vp),
                                  P(c_i64), c_i32, P(lpsift_ransac_params), c_vp, ctypes.c_size_t,
                                  P(c_vp), P(c_vp), P(c_vp), c_vp, c_vp, c_vp]
    lib.lpsift_quantize_u8.restype = ctypes.c_int
    lib.lpsift_quantize_u8.argtypes = [c_vp, c_i64, c_vp, c_vp]
    lib.lpsift_quantize_lowp.restype = ctypes.c_int
    lib.lpsift_quantize_lowp.argtypes = [c_vp, c_i64, c_i32, c_vp, c_vp, c_vp]
    lib.lpsift_match_u8_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_match_u8_workspace_size.argtypes = [c_i64, c_i64]
    lib.lpsift_match_u8.restype = ctypes.c_int
    lib.lpsift_match_u8.argtypes = [c_vp, c_i64, c_vp, c_i64, c_f64, c_f32, c_vp,
                                    ctypes.c_size_t, c_vp, c_vp, c_vp, c_vp]
    lib.lpsift_describe_multi_workspace_size.restype = ctypes.c_size_t
    lib.lpsift_describe_multi_workspace_size.argtypes = [P(lpsift_image), c_i32, P(lpsift_params)]
    lib.lpsift_describe_multi.restype = ctypes.c_int
    lib.lpsift_describe_multi.argtypes = [P(lpsift_image), c_i32, P(lpsift_keypoints),
                                          P(lpsift_params), c_i32, c_f32, c_vp, ctypes.c_size_t,
                                          P(c_vp), P(c_vp), P(c_vp), c_vp, c_vp]
    lib.lpsift_warp_blend.restype = ctypes.c_int
    lib.lpsift_warp_blend.argtypes = [P(lpsift_image), c_i32, c_vp, c_f64, c_f64, c_i32, c_i32,
                                      c_vp, c_vp, c_vp]
    lib.lpsift_probe_out_size.restype = c_i64
    lib.lpsift_probe_out_size.argtypes = []
    lib.lpsift_probe_ops.restype = c_f64
    lib.lpsift_probe_ops.argtypes = [c_i32, c_i64]
    lib.lpsift_probe.restype = ctypes.c_int
    lib.lpsift_probe.argtypes = [c_i32, c_i64, c_vp, c_vp]
    lib.lpsift_ransac_host.restype = ctypes.c_int
    lib.lpsift_refine_host.restype = ctypes.c_int
    lib.lpsift_refine_host.argtypes = [c_vp, c_vp, c_i64, c_f64, c_i32, c_vp, c_vp, c_vp, c_vp]
    lib.lpsift_ransac_host.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i32, c_f64, c_vp, c_vp,
                                       P(c_i64), P(c_i32)]
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().lpsift_status_string(int(status)).decode()


def _check(fn: str, status: int):
    if status != LPSIFT_OK:
        raise LpsiftError(fn, status)


class Params:
    """Window sizes L (Sec. 2.2), descriptor subregions d and beta0 (Eq. 3-4;
    <= 0 picks the largest admissible value)."""

    def __init__(self, L: Sequence[int], d: int = 4, beta0: float = 0.0):
        if not 1 <= len(L) <= MAX_SCALES:
            raise ValueError("1..8 window sizes")
        self.L = [int(v) for v in L]
        self.d = int(d)
        self.beta0 = float(beta0)

    def c(self) -> lpsift_params:
        p = lpsift_params()
        p.n_scales = len(self.L)
        for i, v in enumerate(self.L):
            p.L[i] = v
        p.d = self.d
        p.beta0 = self.beta0
        return p


def num_keypoints(h: int, w: int, params: Params) -> int:
    n = load().lpsift_num_keypoints(h, w, ctypes.byref(params.c()))
    if n < 0:
        raise ValueError("invalid image size or parameters")
    return int(n)


def _stream(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _temp(nbytes: int, dtype, dev, stream):
    """A temporary device buffer used by work enqueued on `stream`: when that
    is not the current stream the block is recorded on it, so that the
    caching allocator does not hand it out again before that work ends."""
    import torch
    t = torch.empty(nbytes, dtype=dtype, device=dev)
    if stream is not None and stream != torch.cuda.current_stream(dev):
        t.record_stream(stream)
    return t


def _image(t) -> lpsift_image:
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.dim() != 2 or not t.is_cuda:
        raise ValueError("images must be 2-D uint8 CUDA tensors")
    if t.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    im = lpsift_image()
    im.data = t.data_ptr()
    im.height, im.width = t.shape
    im.pitch = t.stride(0)
    return im


def _images(images) -> "ctypes.Array":
    arr = (lpsift_image * len(images))()
    for i, t in enumerate(images):
        arr[i] = _image(t)
    return arr


def empty_keypoints(n: int, device) -> Dict[str, "object"]:
    import torch
    return {"x": torch.empty(n, dtype=torch.int32, device=device),
            "y": torch.empty(n, dtype=torch.int32, device=device),
            "scale": torch.empty(n, dtype=torch.uint8, device=device),
            "type": torch.empty(n, dtype=torch.int8, device=device),
            "value": torch.empty(n, dtype=torch.uint8, device=device),
            "contrast": torch.empty(n, dtype=torch.float32, device=device)}


def _kp_struct(kp) -> lpsift_keypoints:
    k = lpsift_keypoints()
    for f in ("x", "y", "scale", "type", "value", "contrast"):
        setattr(k, f, kp[f].data_ptr())
    k.capacity = kp["x"].numel()
    return k


def _kps(kps) -> "ctypes.Array":
    arr = (lpsift_keypoints * len(kps))()
    for i, kp in enumerate(kps):
        arr[i] = _kp_struct(kp)
    return arr


def detect(images, params: Params, out=None, stream=None) -> List[Dict[str, "object"]]:
    """Window maxima and minima of every image at every L (fixed slots)."""
    lib = load()
    imgs = _images(images)
    if out is None:
        out = [empty_keypoints(num_keypoints(t.shape[0], t.shape[1], params), t.device)
               for t in images]
    p = params.c()
    _check("lpsift_detect", lib.lpsift_detect(imgs, len(images), ctypes.byref(p), _kps(out),
                                              _stream(stream)))
    return out


def describe_workspace_size(images, params: Params) -> int:
    return int(load().lpsift_describe_workspace_size(_images(images), len(images),
                                                     ctypes.byref(params.c())))


def describe(images, kps, params: Params, workspace=None, theta=None, desc=None, stream=None):
    """Orientation (radians) and 128-d descriptors of every keypoint slot."""
    import torch
    lib = load()
    imgs = _images(images)
    dev = images[0].device
    n = len(images)
    if theta is None:
        theta = [torch.empty(kp["x"].numel(), dtype=torch.float32, device=dev) for kp in kps]
    if desc is None:
        desc = [torch.empty((kp["x"].numel(), DESC_DIM), dtype=torch.float32, device=dev)
                for kp in kps]
    p = params.c()
    need = int(lib.lpsift_describe_workspace_size(imgs, n, ctypes.byref(p)))
    if workspace is None:
        workspace = _temp(max(need, 1), torch.uint8, dev, stream)
    th = (c_vp * n)(*[t.data_ptr() for t in theta])
    de = (c_vp * n)(*[t.data_ptr() for t in desc])
    _check("lpsift_describe", lib.lpsift_describe(imgs, n, _kps(kps), ctypes.byref(p),
                                                  workspace.data_ptr(), workspace.numel(), th, de,
                                                  _stream(stream)))
    return theta, desc


def match_params(ratio: float = 0.8, abs_thresh: float = math.inf, precision: int = 0,
                 b_chunks: int = 0, stats=None, qblock_waves: int = 0,
                 topk: int = 0) -> lpsift_match_params:
    mp = lpsift_match_params()
    mp.ratio = ratio
    mp.abs_thresh = abs_thresh
    mp.precision = precision
    mp.b_chunks = b_chunks
    mp.qblock_waves = qblock_waves
    mp.topk = topk
    mp.stats = None if stats is None else stats.data_ptr()
    return mp


NOALLOC_SCRATCH_BYTES = 64 << 20     # LPSIFT_NOALLOC_SCRATCH_BYTES


def match_workspace_size(nA: Sequence[int], nB: Sequence[int], mp: lpsift_match_params) -> int:
    n = len(nA)
    return int(load().lpsift_match_workspace_size((c_i64 * n)(*nA), (c_i64 * n)(*nB), n,
                                                  ctypes.byref(mp)))


def _match_args(descA, descB, out, workspace, need, stream=None):
    """Pointer arrays of a match call; a missing workspace (when `need` is
    given) or output is allocated here and tied to `stream`."""
    import torch
    n = len(descA)
    if len(descB) != n or n < 1:
        raise ValueError("descA and descB must be equal-length non-empty lists")
    for t in list(descA) + list(descB):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != DESC_DIM or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError("descriptors must be contiguous float32 CUDA tensors [n, 128]")
    dev = descA[0].device
    nA = [int(t.shape[0]) for t in descA]
    nB = [int(t.shape[0]) for t in descB]
    if workspace is None and need is not None:
        workspace = _temp(max(need(nA, nB), 256), torch.uint8, dev, stream)
    if out is None:
        out = [{"match": torch.empty(a, dtype=torch.int32, device=dev),
                "d1": torch.empty(a, dtype=torch.float32, device=dev),
                "d2": torch.empty(a, dtype=torch.float32, device=dev)} for a in nA]
    ptr = lambda ts: (c_vp * n)(*[t.data_ptr() for t in ts])
    head = (ptr(descA), (c_i64 * n)(*nA), ptr(descB), (c_i64 * n)(*nB), n)
    tail = (0 if workspace is None else workspace.data_ptr(),
            0 if workspace is None else workspace.numel(), ptr([o["match"] for o in out]),
            ptr([o["d1"] for o in out]), ptr([o["d2"] for o in out]))
    return out, head, tail


def match(descA, descB, ratio: float = 0.8, abs_thresh: float = math.inf, precision: int = 0,
          b_chunks: int = 0, workspace=None, out=None, stream=None,
          stats=None, qblock_waves: int = 0, topk: int = 0) -> List[Dict[str, "object"]]:
    """Nearest neighbour of every row of descA[p] among descB[p] with the ratio
    test, for every pair p. stats: optional int32 CUDA tensor [1] that receives
    the number of queries the split path re-matched in FP32 (sum over pairs).
    b_chunks, qblock_waves: the work split (0 = automatic; see match_tune).
    topk: candidates rescored per query at precisions 1 and 2 (0 = 8)."""
    lib = load()
    mp = match_params(ratio, abs_thresh, precision, b_chunks, stats, qblock_waves, topk)
    out, head, tail = _match_args(descA, descB, out, workspace,
                                  lambda nA, nB: match_workspace_size(nA, nB, mp), stream)
    _check("lpsift_match", lib.lpsift_match(*head, ctypes.byref(mp), *tail, _stream(stream)))
    return out


def match_noalloc(descA, descB, ratio: float = 0.8, abs_thresh: float = math.inf,
                  precision: int = 0, b_chunks: int = 0, out=None, stream=None,
                  stats=None, qblock_waves: int = 0, topk: int = 0) -> List[Dict[str, "object"]]:
    """match() through lpsift_match_noalloc: the library's fixed per-device
    scratch array is the workspace, so with `out` given nothing is allocated.
    Calls that overlap on one device race on that array."""
    lib = load()
    mp = match_params(ratio, abs_thresh, precision, b_chunks, stats, qblock_waves, topk)
    out, head, tail = _match_args(descA, descB, out, None, None, stream)
    _check("lpsift_match_noalloc",
           lib.lpsift_match_noalloc(*head, ctypes.byref(mp), *tail[2:], _stream(stream)))
    return out


def quantize_u8(desc, out=None, stream=None):
    """uint8 form of descriptors: min(255, rint(512 d)) per element."""
    import torch
    if desc.dtype != torch.float32 or desc.dim() != 2 or desc.shape[1] != DESC_DIM \
            or not desc.is_cuda or not desc.is_contiguous():
        raise ValueError("descriptors must be contiguous float32 CUDA tensors [n, 128]")
    if out is None:
        out = torch.empty(desc.shape, dtype=torch.uint8, device=desc.device)
    _check("lpsift_quantize_u8", load().lpsift_quantize_u8(desc.data_ptr(), desc.shape[0],
                                                           out.data_ptr(), _stream(stream)))
    return out


def quantize_lowp(desc, precision: int, out=None, scale=None, stream=None):
    """The BF16 (precision 1: int16 bit patterns [n, 128]) or FP8 E4M3
    (precision 2: uint8 codes [n, 128] plus FP32 scales [n]) form of
    descriptors that lpsift_match contracts at that precision. Returns
    (codes, scales or None)."""
    import torch
    if desc.dtype != torch.float32 or desc.dim() != 2 or desc.shape[1] != DESC_DIM \
            or not desc.is_cuda or not desc.is_contiguous():
        raise ValueError("descriptors must be contiguous float32 CUDA tensors [n, 128]")
    if precision not in (1, 2):
        raise ValueError("precision must be 1 (BF16) or 2 (FP8 E4M3)")
    n = desc.shape[0]
    if out is None:
        out = torch.empty((n, DESC_DIM), dtype=torch.int16 if precision == 1 else torch.uint8,
                          device=desc.device)
    if precision == 2 and scale is None:
        scale = torch.empty(n, dtype=torch.float32, device=desc.device)
    _check("lpsift_quantize_lowp", load().lpsift_quantize_lowp(
        desc.data_ptr(), n, precision, out.data_ptr(),
        scale.data_ptr() if precision == 2 else None, _stream(stream)))
    return out, (scale if precision == 2 else None)


def match_u8_workspace_size(nA: int, nB: int) -> int:
    return int(load().lpsift_match_u8_workspace_size(nA, nB))


def match_u8(qA, qB, ratio: float = 0.8, abs_thresh: float = math.inf, workspace=None,
             out=None, stream=None) -> Dict[str, "object"]:
    """Exact nearest neighbour of every row of qA among qB (uint8 [n, 128]
    CUDA tensors) on integer squared distances, with the ratio test; d1, d2 are
    sqrt(D) / 512."""
    import torch
    for t in (qA, qB):
        if t.dtype != torch.uint8 or t.dim() != 2 or t.shape[1] != DESC_DIM or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError("descriptors must be contiguous uint8 CUDA tensors [n, 128]")
    nA, nB = int(qA.shape[0]), int(qB.shape[0])
    dev = qA.device
    if workspace is None:
        workspace = _temp(max(match_u8_workspace_size(nA, nB), 256), torch.uint8, dev, stream)
    if out is None:
        out = {"match": torch.empty(nA, dtype=torch.int32, device=dev),
               "d1": torch.empty(nA, dtype=torch.float32, device=dev),
               "d2": torch.empty(nA, dtype=torch.float32, device=dev)}
    _check("lpsift_match_u8", load().lpsift_match_u8(
        qA.data_ptr(), nA, qB.data_ptr(), nB, ratio, abs_thresh, workspace.data_ptr(),
        workspace.numel(), out["match"].data_ptr(), out["d1"].data_ptr(), out["d2"].data_ptr(),
        _stream(stream)))
    return out


TUNE_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16)


def _bucket(n: int) -> int:
    """Power-of-two bucket of a descriptor count (tuning cache key)."""
    return 0 if n <= 0 else 1 << (int(n) - 1).bit_length()


def match_tune(descA, descB, ratio: float = 0.8, abs_thresh: float = math.inf,
               precision: int = 0, candidates: Sequence[int] = TUNE_CANDIDATES, reps: int = 2,
               cache: Optional[str] = None, stream=None,
               waves: Sequence[int] = (0,)) -> Dict[str, object]:
    """Pick the fastest work split for this set of pairs by timing
    lpsift_match_tune on the device: the candidate-range split (b_chunks, over
    `candidates`) and the FP32 contraction's wavefronts per workgroup
    (qblock_waves, over `waves`; 0 = the default of 4). cache: optional JSON
    file; a result is stored under a key of the device name, precision, pair
    count, power-of-two buckets of the total query and candidate counts and the
    searched values, and reused when the key is present. Returns {"b_chunks",
    "qblock_waves", "ms" ([len(waves)][len(candidates)]), "candidates", "waves",
    "cached"}."""
    import json
    import torch
    cands = [int(c) for c in candidates]
    wv = [int(w) for w in waves]
    key = None
    if cache is not None:
        nq = sum(int(t.shape[0]) for t in descA)
        nc = sum(int(t.shape[0]) for t in descB)
        key = "|".join(str(v) for v in (torch.cuda.get_device_name(descA[0].device), precision,
                                        len(descA), _bucket(nq), _bucket(nc),
                                        ",".join(map(str, cands)), ",".join(map(str, wv))))
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                r = dict(table[key])
                r["cached"] = True
                return r
    lib = load()
    mp = match_params(ratio, abs_thresh, precision, 0, None)

    def need(nA, nB):
        m = match_params(ratio, abs_thresh, precision, 0, None)
        b = 0
        for w in wv:
            m.qblock_waves = w
            for c in cands:
                m.b_chunks = c
                b = max(b, match_workspace_size(nA, nB, m))
        return b
    _, head, tail = _match_args(descA, descB, None, None, need, stream)
    k, nw = len(cands), len(wv)
    ms = (c_f32 * (k * nw))()
    best, best_w = c_i32(0), c_i32(0)
    _check("lpsift_match_tune", lib.lpsift_match_tune(
        *head, ctypes.byref(mp), (c_i32 * k)(*cands), k, (c_i32 * nw)(*wv), nw, int(reps),
        *tail, ms, ctypes.byref(best), ctypes.byref(best_w), _stream(stream)))
    r = {"b_chunks": int(best.value), "qblock_waves": int(best_w.value),
         "ms": [[float(ms[w * k + c]) for c in range(k)] for w in range(nw)],
         "candidates": cands, "waves": wv, "cached": False}
    if cache is not None:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = {k_: v for k_, v in r.items() if k_ != "cached"}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return r


KERNELS = ("detect", "gradient", "describe", "match_norms", "match_fp32", "match_split",
           "match_rescore", "match_rematch", "match_lowp", "score", "prune", "train", "ransac",
           "match_u8", "match_u8_aux", "orient_multi", "warp")
SCORER_PARAMS = 20801


def describe_selected(images, kps, params: Params, sel, workspace=None, theta=None, desc=None,
                      stream=None):
    """Orientation and descriptor of the listed slots sel[i] (int32 CUDA
    tensors) of each image, compacted in list order."""
    import torch
    lib = load()
    imgs = _images(images)
    dev = images[0].device
    n = len(images)
    ns = [int(s.numel()) for s in sel]
    if theta is None:
        theta = [torch.empty(m, dtype=torch.float32, device=dev) for m in ns]
    if desc is None:
        desc = [torch.empty((m, DESC_DIM), dtype=torch.float32, device=dev) for m in ns]
    p = params.c()
    need = int(lib.lpsift_describe_workspace_size(imgs, n, ctypes.byref(p)))
    if workspace is None:
        workspace = _temp(max(need, 1), torch.uint8, dev, stream)
    _check("lpsift_describe_selected", lib.lpsift_describe_selected(
        imgs, n, _kps(kps), ctypes.byref(p), (c_vp * n)(*[s.data_ptr() for s in sel]),
        (c_i64 * n)(*ns), workspace.data_ptr(), workspace.numel(),
        (c_vp * n)(*[t.data_ptr() for t in theta]), (c_vp * n)(*[t.data_ptr() for t in desc]),
        _stream(stream)))
    return theta, desc


def describe_multi_workspace_size(images, params: Params) -> int:
    return int(load().lpsift_describe_multi_workspace_size(_images(images), len(images),
                                                           ctypes.byref(params.c())))


def describe_multi(images, kps, params: Params, max_orient: int = 4, peak_ratio: float = 0.8,
                   workspace=None, out=None, stream=None):
    """Multi-orientation rows of every keypoint slot (dominant orientation
    first, then the secondary peaks): per image a dict with rows (slot of each
    row), theta, desc (capacity n_kp * max_orient rows) and n_rows, a device
    int64 tensor [n_images] with the row counts (read it to trim)."""
    import torch
    lib = load()
    ims = _images(images)
    n = len(images)
    P = params.c()
    dev = images[0].device
    if workspace is None:
        workspace = _temp(max(describe_multi_workspace_size(images, params), 256), torch.uint8,
                          dev, stream)
    if out is None:
        caps = [int(k["x"].numel()) * max_orient for k in kps]
        out = {"rows": [torch.empty(c, dtype=torch.int32, device=dev) for c in caps],
               "theta": [torch.empty(c, dtype=torch.float32, device=dev) for c in caps],
               "desc": [torch.empty((c, DESC_DIM), dtype=torch.float32, device=dev) for c in caps],
               "n_rows": torch.zeros(n, dtype=torch.int64, device=dev)}
    ptr = lambda ts: (c_vp * n)(*[t.data_ptr() for t in ts])
    _check("lpsift_describe_multi", lib.lpsift_describe_multi(
        ims, n, _kps(kps), ctypes.byref(P), max_orient, peak_ratio, workspace.data_ptr(),
        workspace.numel(), ptr(out["rows"]), ptr(out["theta"]), ptr(out["desc"]),
        out["n_rows"].data_ptr(), _stream(stream)))
    return out


def score(images, kps, params: Params, weights, out=None, stream=None):
    """Scorer logits of every keypoint slot (weights: FP32 CUDA tensor [20801])."""
    import torch
    lib = load()
    n = len(images)
    if weights.dtype != torch.float32 or weights.numel() != SCORER_PARAMS or not weights.is_cuda:
        raise ValueError("weights must be a float32 CUDA tensor of 20801 values")
    if out is None:
        out = [torch.empty(kp["x"].numel(), dtype=torch.float32, device=weights.device)
               for kp in kps]
    _check("lpsift_score", lib.lpsift_score(
        _images(images), n, _kps(kps), ctypes.byref(params.c()), weights.data_ptr(),
        (c_vp * n)(*[t.data_ptr() for t in out]), _stream(stream)))
    return out


def keep_count(n: int, num: int = 3, den: int = 10) -> int:
    """ceil(n num / den) in integers (30 % by default)."""
    return -(-int(n) * num // den)


def prune(scores, k: Sequence[int], out=None, stream=None):
    """Ascending slots of the k[i] best scores of each image (int32 tensors)."""
    import torch
    lib = load()
    n = len(scores)
    if out is None:
        out = [torch.empty(int(kk), dtype=torch.int32, device=s.device) for s, kk in zip(scores, k)]
    _check("lpsift_prune", lib.lpsift_prune(
        (c_vp * n)(*[s.data_ptr() for s in scores]), (c_i64 * n)(*[s.numel() for s in scores]),
        (c_i64 * n)(*[int(x) for x in k]), n, (c_vp * n)(*[t.data_ptr() for t in out]),
        _stream(stream)))
    return out


def scorer_gather(images, kps, params: Params, sel=None, stream=None):
    """uint8 patches [m, 256] and float extras [m, 2] of listed (or all) slots."""
    import torch
    lib = load()
    n = len(images)
    dev = images[0].device
    ms = [int(s.numel()) for s in sel] if sel is not None else \
        [num_keypoints(t.shape[0], t.shape[1], params) for t in images]
    patches = [torch.empty((m, 256), dtype=torch.uint8, device=dev) for m in ms]
    extra = [torch.empty((m, 2), dtype=torch.float32, device=dev) for m in ms]
    sel_arr = None if sel is None else (c_vp * n)(*[s.data_ptr() for s in sel])
    n_arr = None if sel is None else (c_i64 * n)(*ms)
    _check("lpsift_scorer_gather", lib.lpsift_scorer_gather(
        _images(images), n, _kps(kps), ctypes.byref(params.c()), sel_arr, n_arr,
        (c_vp * n)(*[t.data_ptr() for t in patches]), (c_vp * n)(*[t.data_ptr() for t in extra]),
        _stream(stream)))
    return patches, extra


class ScorerTrainer:
    """Device state of scorer training: FP32 weights, Adam moments, workspace."""

    def __init__(self, weights, batch: int):
        import torch
        self.weights = weights
        self.m = torch.zeros_like(weights)
        self.v = torch.zeros_like(weights)
        self.batch = int(batch)
        need = int(load().lpsift_scorer_train_workspace_size(self.batch))
        self.ws = torch.empty(max(need, 4), dtype=torch.uint8, device=weights.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=weights.device)
        self.t = 0

    def step(self, patches, extra, labels, cweight, lr: float, stream=None):
        """One Adam step on a batch (<= the batch size given at construction);
        self.loss holds the batch loss before the step."""
        b = int(labels.numel())
        if b > self.batch:
            raise ValueError("batch larger than the trainer's workspace")
        self.t += 1
        _check("lpsift_scorer_train_step", load().lpsift_scorer_train_step(
            patches.data_ptr(), extra.data_ptr(), labels.data_ptr(), cweight.data_ptr(), b,
            self.weights.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.t, float(lr),
            self.ws.data_ptr(), self.ws.numel(), self.loss.data_ptr(), _stream(stream)))


def timing_enable(on: bool = True):
    """Reset the per-kernel timing sums and switch timing on or off."""
    _check("lpsift_timing_enable", load().lpsift_timing_enable(1 if on else 0))


def timing_read() -> Dict[str, Dict[str, float]]:
    """{kernel: {"ms": summed device ms, "launches": n}} since the last reset
    (waits for the recorded events)."""
    lib = load()
    out = {}
    for k, name in enumerate(KERNELS):
        ms, n = c_f64(0.0), c_i64(0)
        _check("lpsift_timing_read", lib.lpsift_timing_read(k, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = {"ms": ms.value, "launches": int(n.value)}
    return out


def features(images, params: Params, stream=None):
    """detect + describe: returns (keypoints, theta, desc), lists per image."""
    kps = detect(images, params, stream=stream)
    theta, desc = describe(images, kps, params, stream=stream)
    return kps, theta, desc


def ransac_gpu(kpA, kpB, matches, uniforms, thresh: float = 3.0, selA=None, selB=None,
               workspace=None, stream=None, out=None):
    """Batched RANSAC on the device for match lists of lpsift_match.
    kpA, kpB: keypoint dicts per pair; matches: int32 tensors [nq]; uniforms:
    float64 CUDA tensor [n_iter, 4, tries]; selA / selB: optional int32 slot
    lists per pair. Returns {"H": [n, 9] float64, "stats": [n, 3] int32
    (matches, inliers, best hypothesis), "slotA", "slotB", "inlier"} (the
    per-pair lists hold stats[p, 0] valid entries)."""
    import torch
    lib = load()
    n = len(matches)
    dev = matches[0].device
    if uniforms.dtype != torch.float64 or uniforms.dim() != 3 or uniforms.shape[1] != 4 \
            or not uniforms.is_contiguous():
        raise ValueError("uniforms must be a contiguous float64 tensor [n_iter, 4, tries]")
    nq = [int(m.numel()) for m in matches]
    rp = lpsift_ransac_params()
    rp.n_iter, rp.tries, rp.thresh = int(uniforms.shape[0]), int(uniforms.shape[2]), float(thresh)
    rp.uniforms = uniforms.data_ptr()
    need = int(lib.lpsift_ransac_workspace_size((c_i64 * n)(*nq), n, rp.n_iter))
    if workspace is None:
        workspace = _temp(max(need, 256), torch.uint8, dev, stream)
    if out is None:
        out = {"slotA": [torch.empty(q, dtype=torch.int32, device=dev) for q in nq],
               "slotB": [torch.empty(q, dtype=torch.int32, device=dev) for q in nq],
               "inlier": [torch.empty(q, dtype=torch.uint8, device=dev) for q in nq],
               "H": torch.zeros((n, 9), dtype=torch.float64, device=dev),
               "stats": torch.zeros((n, 3), dtype=torch.int32, device=dev)}
    slotA, slotB, inl, H, stats = out["slotA"], out["slotB"], out["inlier"], out["H"], out["stats"]
    ptr = lambda ts: (c_vp * n)(*[t.data_ptr() for t in ts])
    _check("lpsift_ransac", lib.lpsift_ransac(
        _kps(kpA), _kps(kpB), None if selA is None else ptr(selA),
        None if selB is None else ptr(selB), ptr(matches), (c_i64 * n)(*nq), n, ctypes.byref(rp),
        workspace.data_ptr(), workspace.numel(), ptr(slotA), ptr(slotB), ptr(inl), H.data_ptr(),
        stats.data_ptr(), _stream(stream)))
    return out


def warp_blend(images, G, x0: float, y0: float, width: int, height: int, canvas=None,
               count=None, with_count: bool = True, stream=None):
    """Blend registered images (uint8 CUDA tensors) into a width x height
    float canvas whose pixel (0, 0) is reference point (x0, y0); G: one 3x3
    transform (image -> reference pixels) per image. Returns (canvas, count)."""
    import numpy as np
    import torch
    n = len(images)
    g = np.ascontiguousarray(np.stack([np.asarray(t, np.float64).reshape(9) for t in G]))
    if g.shape != (n, 9):
        raise ValueError("one 3x3 transform per image")
    dev = images[0].device
    if canvas is None:
        canvas = torch.empty((height, width), dtype=torch.float32, device=dev)
    if count is None and with_count:
        count = torch.empty((height, width), dtype=torch.uint8, device=dev)
    _check("lpsift_warp_blend", load().lpsift_warp_blend(
        _images(images), n, g.ctypes.data, float(x0), float(y0), int(width), int(height),
        canvas.data_ptr(), None if count is None else count.data_ptr(), _stream(stream)))
    return canvas, count


PROBES = {"fp32": 0, "bf16": 1, "fp8": 2, "int8": 3}


def mfma_probe(kind: str, iters: int = 4096, reps: int = 3, device=None) -> float:
    """Achieved matrix-core rate (TFLOP/s or TOP/s) of the probe kernel of one
    precision: the best of `reps` timed calls after one untimed call."""
    import torch
    lib = load()
    k = PROBES[kind]
    dev = device or torch.device("cuda:0")
    out = torch.empty(int(lib.lpsift_probe_out_size()), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    _check("lpsift_probe", lib.lpsift_probe(k, iters, out.data_ptr(), stream.cuda_stream))
    best = math.inf
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        _check("lpsift_probe", lib.lpsift_probe(k, iters, out.data_ptr(), stream.cuda_stream))
        e[1].record(stream)
        torch.cuda.synchronize(dev)
        best = min(best, e[0].elapsed_time(e[1]))
    return float(lib.lpsift_probe_ops(k, iters)) / (best * 1e-3) / 1e12


def ransac(xyA, xyB, samples, thresh: float = 3.0):
    """Homography A -> B from matched pairs by RANSAC on the host (FP64).
    xyA, xyB: [n, 2] arrays; samples: [n_iter, 4] int indices (the random
    draws). Returns (H [3, 3] or None, inlier mask [n] bool, best iteration)."""
    import numpy as np
    lib = load()
    a = np.ascontiguousarray(xyA, dtype=np.float64).reshape(-1, 2)
    b = np.ascontiguousarray(xyB, dtype=np.float64).reshape(-1, 2)
    if a.shape != b.shape:
        raise ValueError("xyA and xyB must have the same shape")
    smp = np.ascontiguousarray(samples, dtype=np.int32).reshape(-1, 4)
    H = np.zeros(9, np.float64)
    mask = np.zeros(len(a), np.uint8)
    n_in, best = c_i64(), c_i32()
    _check("lpsift_ransac_host", lib.lpsift_ransac_host(
        a.ctypes.data, b.ctypes.data, len(a), smp.ctypes.data, len(smp), float(thresh),
        H.ctypes.data, mask.ctypes.data, ctypes.byref(n_in), ctypes.byref(best)))
    return (H.reshape(3, 3) if best.value >= 0 else None), mask.astype(bool), best.value


def refine_homography(xyA, xyB, H, thresh: float = 3.0, max_rounds: int = 20):
    """Least-squares rounds over the inliers of H until the inlier set stops
    changing (host, FP64). Returns (H [3, 3], inlier mask [n] bool, rounds)."""
    import numpy as np
    lib = load()
    a = np.ascontiguousarray(xyA, dtype=np.float64).reshape(-1, 2)
    b = np.ascontiguousarray(xyB, dtype=np.float64).reshape(-1, 2)
    if a.shape != b.shape:
        raise ValueError("xyA and xyB must have the same shape")
    G = np.ascontiguousarray(H, dtype=np.float64).reshape(9).copy()
    mask = np.zeros(len(a), np.uint8)
    n_in, rounds = c_i64(), c_i32()
    _check("lpsift_refine_host", lib.lpsift_refine_host(
        a.ctypes.data, b.ctypes.data, len(a), float(thresh), int(max_rounds), G.ctypes.data,
        mask.ctypes.data, ctypes.byref(n_in), ctypes.byref(rounds)))
    return G.reshape(3, 3), mask.astype(bool), rounds.value
