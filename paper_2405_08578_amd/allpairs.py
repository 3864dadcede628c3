"""All-pairs feature matching of an image set (the mosaic workload of Sec. 4:
every image matched against every other before the homographies are solved).

AllPairs preallocates every buffer once for a fixed list of images — keypoint
slots, orientations, descriptors, both workspaces and the match lists of the
N (N - 1) / 2 pairs (i < j, image i as queries, image j as registered set) —
so that one step is three library calls (detect, describe, match) that
allocate nothing and never synchronise. The step can run eagerly or be
captured once into a HIP graph (torch.cuda.CUDAGraph) and replayed: the
launch sequence is fixed by the image shapes, and replays read the images from
the same device buffers. Optionally the step ends with the batched GPU RANSAC
of every pair (the pairwise homographies of the mosaic, Sec. 4). With
u8=True the match stage quantises every descriptor set to uint8 and runs the
exact integer matcher on each pair (one workspace, reused pair after pair on
the stream).
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

from . import (DESC_DIM, Params, describe, describe_workspace_size, detect, empty_keypoints,
               load, match, match_params, match_u8, match_u8_workspace_size,
               match_workspace_size, num_keypoints, quantize_u8, ransac_gpu)


def pair_list(n: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


class AllPairs:
    def __init__(self, images, params: Params, precision: int = 0, b_chunks: int = 0,
                 ratio: float = 0.8, abs_thresh: float = math.inf, ransac_uniforms=None,
                 ransac_thresh: float = 3.0, u8: bool = False, qblock_waves: int = 0):
        """ransac_uniforms: optional float64 CUDA tensor [n_iter, 4, tries];
        when given, every step ends with the batched GPU RANSAC of all pairs
        (self.ransac: H [pairs, 9], stats [pairs, 3], slot and inlier lists)."""
        import torch
        if len(images) < 2:
            raise ValueError("need at least two images")
        self.images = list(images)
        self.params = params
        self.precision = precision
        self.b_chunks = b_chunks
        self.qblock_waves = qblock_waves
        self.ratio = ratio
        self.abs_thresh = abs_thresh
        dev = self.images[0].device
        self.device = dev
        self.pairs = pair_list(len(self.images))
        self.n_kp = [num_keypoints(t.shape[0], t.shape[1], params) for t in self.images]
        self.kps = [empty_keypoints(n, dev) for n in self.n_kp]
        self.theta = [torch.empty(n, dtype=torch.float32, device=dev) for n in self.n_kp]
        self.desc = [torch.empty((n, DESC_DIM), dtype=torch.float32, device=dev)
                     for n in self.n_kp]
        self.dws = torch.empty(max(describe_workspace_size(self.images, params), 256),
                               dtype=torch.uint8, device=dev)
        self.stats = torch.zeros(1, dtype=torch.int32, device=dev)
        self.u8 = u8
        if u8:
            self.q = [torch.empty((n, DESC_DIM), dtype=torch.uint8, device=dev) for n in self.n_kp]
            need = max(match_u8_workspace_size(self.n_kp[i], self.n_kp[j]) for i, j in self.pairs)
        else:
            mp = match_params(ratio, abs_thresh, precision, b_chunks, None, qblock_waves)
            need = match_workspace_size([self.n_kp[i] for i, _ in self.pairs],
                                        [self.n_kp[j] for _, j in self.pairs], mp)
        self.mws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        self.out = [{"match": torch.empty(self.n_kp[i], dtype=torch.int32, device=dev),
                     "d1": torch.empty(self.n_kp[i], dtype=torch.float32, device=dev),
                     "d2": torch.empty(self.n_kp[i], dtype=torch.float32, device=dev)}
                    for i, _ in self.pairs]
        self.graph = None
        self.ransac = None
        self.ransac_uniforms = ransac_uniforms
        self.ransac_thresh = ransac_thresh
        if ransac_uniforms is not None:
            import ctypes
            nq = [self.n_kp[i] for i, _ in self.pairs]
            n = len(nq)
            need = int(load().lpsift_ransac_workspace_size((ctypes.c_int64 * n)(*nq), n,
                                                           int(ransac_uniforms.shape[0])))
            self.rws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)

    @property
    def megapixels(self) -> float:
        return sum(t.shape[0] * t.shape[1] for t in self.images) / 1e6

    def run(self, stream=None):
        """Enqueue one step on `stream` (default: the current stream)."""
        detect(self.images, self.params, out=self.kps, stream=stream)
        describe(self.images, self.kps, self.params, workspace=self.dws, theta=self.theta,
                 desc=self.desc, stream=stream)
        if self.u8:
            for d, q in zip(self.desc, self.q):
                quantize_u8(d, out=q, stream=stream)
            for (i, j), o in zip(self.pairs, self.out):
                match_u8(self.q[i], self.q[j], ratio=self.ratio, abs_thresh=self.abs_thresh,
                         workspace=self.mws, out=o, stream=stream)
        else:
            match([self.desc[i] for i, _ in self.pairs], [self.desc[j] for _, j in self.pairs],
                  ratio=self.ratio, abs_thresh=self.abs_thresh, precision=self.precision,
                  b_chunks=self.b_chunks, workspace=self.mws, out=self.out, stream=stream,
                  stats=self.stats, qblock_waves=self.qblock_waves)
        if self.ransac_uniforms is not None:
            self.ransac = ransac_gpu([self.kps[i] for i, _ in self.pairs],
                                     [self.kps[j] for _, j in self.pairs],
                                     [o["match"] for o in self.out], self.ransac_uniforms,
                                     self.ransac_thresh, workspace=self.rws, stream=stream,
                                     out=self.ransac)

    def capture(self, warmup: int = 1):
        """Capture one step into a graph (after `warmup` eager steps on a side
        stream, as graph capture requires)."""
        import torch
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
