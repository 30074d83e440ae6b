"""The paper's own fusion outcome as a fixture (tests/golden/table4_fusion.json).

Sec. VII runs six kernels in order (Table II types, Table IV dependence
types) and reports the fusion the partition model produced: the first five
kernels form one fused kernel and the Kalman filter, the only kernel-to-kernel
dependence, stays alone; a hand-made two-group split of the first five is its
non-optimal comparison.  Both the brute-force partition oracle (under the
Eq. 1 / Eq. 2 traffic model) and the library's planner (through the C ABI,
host only) must reproduce that outcome.

The library's generic stages stand in for the six kernels: point stages for
the thread-to-thread kernels, weighted stencils of radius 2 and 1 for the
Gaussian and gradient filters, and a point stage with a kernel-to-kernel
dependence for the Kalman filter.  The IIR filter's use of earlier frames has
no generic-stage form; the partition depends only on the dependence types and
the bytes, which the stand-ins keep.
"""
import json
import math
import os

import numpy as np

from oracle import partition as P
from paper_1509_04394_amd import fz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_fusion.json")


def _fixture():
    with open(GOLDEN) as f:
        return json.load(f)


def _groups(pairs):
    return [tuple(p) for p in pairs]


def test_fixture_shape():
    g = _fixture()
    assert [k["dep"] for k in g["kernels"]] == ["TT", "TT", "TMT", "TMT", "TT", "KK"]
    for split in ("full_fusion", "two_fusion"):  # exact covers, in order
        covered = [i for a, b in g[split] for i in range(a, b + 1)]
        assert covered == list(range(len(g["kernels"])))


def test_partition_oracle_reproduces_full_fusion():
    g = _fixture()
    n = len(g["kernels"])
    # bytes per pixel: RGBA u8 in, gray and filtered frames as f32, two gradient
    # channels, a thresholded f32 frame, and the tracker's f32 output
    bi = [4, 4, 4, 4, 8, 4]
    bo = [4, 4, 4, 8, 4, 4]
    kk = [k["dep"] == "KK" for k in g["kernels"]]
    c = [[None] * n for _ in range(n)]
    for a in range(n):
        for b in range(a, n):
            # a kernel-to-kernel dependence inside a group makes it infeasible (Sec. VI-A)
            c[a][b] = math.inf if any(kk[j] for j in range(a + 1, b + 1)) else P.compulsory_bytes(bi, bo, a, b)
    total, groups = P.best(c, n)
    assert groups == _groups(g["full_fusion"])
    two = sum(c[a][b] for a, b in g["two_fusion"])
    assert total < two < P.unfused_bytes(bi, bo)


def _stand_in_chain():
    gauss = np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1]).astype(np.float32) / 256.0
    grad = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], np.float32)
    return [
        ("point", "affine", 0.25, 0.0),    # K1: RGBA to gray (thread to thread)
        ("point", "affine", 0.9, 1.0),     # K2: IIR filter (thread to thread)
        ("stencil", 2, 2, gauss),          # K3: Gaussian smoothing (thread to multi-thread)
        ("stencil", 1, 1, grad),           # K4: gradient filter (thread to multi-thread)
        ("point", "clamp", 0.0, 255.0),    # K5: threshold (thread to thread)
        ("point", "abs", 0.0, 0.0),        # K6: Kalman filter (kernel to kernel)
    ]


def test_planner_reproduces_full_fusion():
    g = _fixture()
    kk = {i: fz.FZ_DEP_KK for i, k in enumerate(g["kernels"]) if k["dep"] == "KK"}
    W, H, T = 432, 192, 1000  # the paper's recorded frame size and frame count
    plan = fz.Plan(_stand_in_chain(), W, H, T, deps=kk)
    assert plan.segments == [b for _, b in g["full_fusion"]]
    two = fz.Plan(_stand_in_chain(), W, H, T, deps=kk, partition=[b for _, b in g["two_fusion"][:-1]])
    assert two.segments == [b for _, b in g["two_fusion"]]
    unfused = fz.Plan(_stand_in_chain(), W, H, T, deps=kk, partition="unfused")
    assert plan.cost < two.cost < unfused.cost
