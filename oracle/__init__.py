"""CPU reference ("oracle") of the video kernel chain -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
use this package.  It imports nothing from the GPU library and the GPU library
never imports it.

* ``chain``: the plain, unfused, frame-by-frame FP64 chain (``oracle.c``),
  Sec. III composition I_out = K_n(...K_1(I_in)).
* ``gchain``: the same for a chain of generic single-channel stages (point,
  weighted stencil, window sum; the Table I classes with free parameters).
* ``partition``: brute-force enumeration of every contiguous partition of a
  kernel sequence (Sec. VI, Fig. 5 model).
* ``mlp``: FP64 forward / backward of the cost-model network.
* ``track``: Kalman tracking of feature points (``track.c``), the stage the
  paper applies after the chain (Sec. III, Table II).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OPS = {
    "rgb2gray": 1, "gauss5": 2, "sobel3": 3, "gradmag": 4, "products": 5,
    "boxsum5": 6, "harris": 7, "threshold": 8, "nms3": 9, "framediff": 10,
}
_IN_CH = {"rgb2gray": 3, "sobel3": 1, "gradmag": 2, "products": 2, "harris": 3}
_OUT_CH = {"sobel3": 2, "products": 3}

SIGMA = 1.0
HARRIS_K = 0.04
THRESHOLD = 1.0e8


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "track.c"),
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        d = ctypes.POINTER(ctypes.c_double)
        lib.or_chain.restype = ctypes.c_int
        lib.or_chain.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, d, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, d, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, d, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        i32 = ctypes.POINTER(ctypes.c_int32)
        lib.or_gchain.restype = ctypes.c_int
        lib.or_gchain.argtypes = [i32, i32, i32, i32, d, d, d, ctypes.c_int32, d, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, d, ctypes.c_int32]
        lib.or_gchain_seq.restype = ctypes.c_int
        lib.or_gchain_seq.argtypes = [i32, i32, i32, i32, i32, d, d, d, ctypes.c_int32, d, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, d]
        lib.or_track.restype = ctypes.c_int64
        lib.or_track.argtypes = [i32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int32, ctypes.c_double, i32, d, ctypes.c_int64]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def chain_channels(ops, in_ch=None):
    """(input channels, output channels) of a chain of op names."""
    ch = _IN_CH.get(ops[0], in_ch if in_ch is not None else 1)
    first = ch
    for op in ops:
        ch = _OUT_CH.get(op, ch if op == "boxsum5" else 1)
    return first, ch


def to_planes(ops, volume):
    """The chain's input as contiguous float64 planes [C][T][H][W] (the
    oracle's own layout): [T][H][W] one channel, [T][H][W][3] RGB interleaved
    for a chain starting with rgb2gray, or [C][T][H][W] planar."""
    v = np.asarray(volume)
    if ops[0] == "rgb2gray":
        return np.ascontiguousarray(np.moveaxis(v, -1, 0), dtype=np.float64)
    if v.ndim == 3:
        return np.ascontiguousarray(v[None], dtype=np.float64)
    return np.ascontiguousarray(v, dtype=np.float64)


def chain(ops, volume, in_ch=None, sigma=SIGMA, k=HARRIS_K, thr=THRESHOLD,
          nthreads=None, max_points=1 << 18):
    """Run the chain ``ops`` (list of names) over ``volume``.

    ``volume`` is [T][H][W] (one channel), [T][H][W][3] (RGB interleaved, for a
    chain starting with rgb2gray) or [C][T][H][W] planar float for multi-channel
    float input.  Returns (out [C][T][H][W] float64, points [n][4] float64 rows
    (t, y, x, response)).
    """
    ops = list(ops)
    return chain_planes(ops, to_planes(ops, volume), sigma, k, thr, nthreads, max_points)


def chain_planes(ops, planes, sigma=SIGMA, k=HARRIS_K, thr=THRESHOLD, nthreads=None, max_points=1 << 18):
    """``chain`` on input already in the oracle's layout (``to_planes``)."""
    ops = list(ops)
    if planes.dtype != np.float64 or not planes.flags.c_contiguous or planes.ndim != 4:
        raise ValueError("planes must be contiguous float64 [C][T][H][W]")
    cin, cout = chain_channels(ops, planes.shape[0])
    if planes.shape[0] != cin:
        raise ValueError(f"chain {ops} wants {cin} input channels, got {planes.shape[0]}")
    C, T, H, W = planes.shape
    out = np.zeros((cout, T, H, W), np.float64)
    codes = (ctypes.c_int32 * len(ops))(*[OPS[o] for o in ops])
    cap = int(max_points)
    pts = np.zeros((max(cap, 1), 4), np.float64)
    npts = ctypes.c_int64(0)
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, T)
    rc = _load().or_chain(codes, len(ops), _dp(planes), C, W, H, T, _dp(out), cout,
                          sigma, k, thr, _dp(pts), cap, ctypes.byref(npts), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle chain failed with code {rc}")
    n = npts.value
    if n > cap:
        raise RuntimeError(f"oracle point buffer overflow ({n} > {cap})")
    return out, pts[:n].copy()


GKINDS = {"point": 0, "stencil": 1, "box": 2, "iir": 3}
POINT_KINDS = {"affine": 0, "abs": 1, "square": 2, "sqrtabs": 3, "clamp": 4}


def _temporal(stages):
    return any(st[0] == "iir" or (st[0] == "stencil" and np.asarray(st[3]).ndim == 3) for st in stages)


def gchain(stages, volume, nthreads=None):
    """Run a generic chain over ``volume`` [T][H][W] (any real dtype).

    ``stages`` is a list of tuples:
      ("point", kind, a, b)       kind in POINT_KINDS; affine is a*v + b,
                                  clamp is min(max(v, a), b)
      ("stencil", rx, ry, w)      w has shape (2ry+1, 2rx+1): correlation
                                  weights, w[v+ry][u+rx] multiplies in(x+u, y+v);
                                  or shape (rt+1, 2ry+1, 2rx+1): a spatio-temporal
                                  stencil, w[tau] multiplies frame t - tau
                                  (frames before the first are the first)
      ("box", rx, ry)             unweighted (2rx+1) x (2ry+1) window sum
      ("iir", a)                  y[t] = a x[t] + (1 - a) y[t-1], y[-1] = x[0]
    Window stages clamp their reads to the frame (replicate borders).  Returns
    out [T][H][W] float64.  Chains with a frame window or an IIR stage run
    stage by stage over the whole volume (or_gchain_seq); the others frame by
    frame (or_gchain).
    """
    v = np.ascontiguousarray(np.asarray(volume), dtype=np.float64)
    if v.ndim != 3:
        raise ValueError("volume must be [T][H][W]")
    T, H, W = v.shape
    n = len(stages)
    kind = (ctypes.c_int32 * n)()
    rx = (ctypes.c_int32 * n)()
    ry = (ctypes.c_int32 * n)()
    rt = (ctypes.c_int32 * n)()
    pk = (ctypes.c_int32 * n)()
    pa = np.zeros(n, np.float64)
    pb = np.zeros(n, np.float64)
    ws = []
    for i, st in enumerate(stages):
        kind[i] = GKINDS[st[0]]
        if st[0] == "point":
            pk[i] = POINT_KINDS[st[1]]
            pa[i] = st[2] if len(st) > 2 else 0.0
            pb[i] = st[3] if len(st) > 3 else 0.0
        elif st[0] == "iir":
            pa[i] = float(st[1])
        else:
            rx[i], ry[i] = int(st[1]), int(st[2])
            if st[0] == "stencil":
                w = np.asarray(st[3], np.float64)
                if w.ndim == 2:
                    w = w[None]
                rt[i] = w.shape[0] - 1
                if w.shape[1:] != (2 * ry[i] + 1, 2 * rx[i] + 1):
                    raise ValueError(f"stage {i}: weights must have shape {(2 * ry[i] + 1, 2 * rx[i] + 1)} "
                                     f"per frame")
                ws.append(w.ravel())
    wcat = np.ascontiguousarray(np.concatenate(ws) if ws else np.zeros(1), dtype=np.float64)
    out = np.zeros_like(v)
    if _temporal(stages):
        rc = _load().or_gchain_seq(kind, rx, ry, rt, pk, _dp(pa), _dp(pb), _dp(wcat), n, _dp(v), W, H, T, _dp(out))
    else:
        if nthreads is None:
            nthreads = min(os.cpu_count() or 1, T)
        rc = _load().or_gchain(kind, rx, ry, pk, _dp(pa), _dp(pb), _dp(wcat), n, _dp(v), W, H, T, _dp(out),
                               int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle generic chain failed with code {rc}")
    return out


# ---------------------------------------------------------------- tracking
TRACK_DEFAULTS = dict(q=0.5, r=1.0, gate=9.21, v0=4.0, max_miss=3)


def track(points, T, q=0.5, r=1.0, gate=9.21, max_miss=3, v0=4.0):
    """Kalman tracking of feature points (``track.c``): points [n][>=3] rows
    (t, y, x, ...) in any order, frames 0..T-1.  Returns (ints [m][3] rows
    (t, id, status), states [m][4] rows (x, y, vx, vy)), one row per live
    track and frame, ordered by frame, then by id (status 0 predicted only,
    1 updated, 2 started)."""
    lib = _load()
    p = np.ascontiguousarray(np.asarray(points)[:, :3], dtype=np.int32) if len(points) else np.zeros((0, 3), np.int32)
    cap = max(1, 4 * len(p) * (max_miss + 2) + 16)
    oi = np.zeros((cap, 3), np.int32)
    od = np.zeros((cap, 4), np.float64)
    i32 = ctypes.POINTER(ctypes.c_int32)
    n = lib.or_track(p.ctypes.data_as(i32), len(p), int(T), float(q), float(r), float(gate), int(max_miss),
                     float(v0), oi.ctypes.data_as(i32), _dp(od), cap)
    if n < 0:
        raise RuntimeError(f"oracle tracker failed with code {n}")
    if n > cap:
        raise RuntimeError("oracle tracker output overflow")
    return oi[:n].copy(), od[:n].copy()
