"""Python binding of the fz C ABI (include/fz.h).

Argument marshalling only: every step of the chain runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  The functions keep
the C names; ``Plan`` is a small convenience wrapper that allocates outputs,
workspace and the point buffer as torch tensors.

The library is loaded from ``libfz.so`` next to this file; if it is missing the
import of any entry point raises (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfz.so")

FZ_OK, FZ_E_INVALID, FZ_E_LDS, FZ_E_HIP, FZ_E_WORKSPACE, FZ_E_UNSUPPORTED = range(6)
FZ_U8, FZ_F32 = 1, 2
FZ_DEP_TT, FZ_DEP_TMT, FZ_DEP_KK = 0, 1, 2
FZ_PART_OPTIMAL, FZ_PART_UNFUSED, FZ_PART_EXPLICIT = 0, 1, 2
FZ_COST_ANALYTIC, FZ_COST_LEARNED, FZ_COST_MEASURED = 0, 1, 2
FZ_ENGINE_AUTO, FZ_ENGINE_TILE, FZ_ENGINE_ROW, FZ_ENGINE_STREAM, FZ_ENGINE_JIT = 0, 1, 2, 3, 4
ENGINES = {"auto": FZ_ENGINE_AUTO, "tile": FZ_ENGINE_TILE, "row": FZ_ENGINE_ROW, "jit": FZ_ENGINE_JIT}
JIT_TILES = [(16, 16), (32, 16), (32, 32), (64, 16), (64, 32)]
FZ_TRACK_MAX_TRACKS = 4096
FZ_TRACK_TOO_MANY_POINTS, FZ_TRACK_TOO_MANY_CANDIDATES, FZ_TRACK_TOO_MANY_TRACKS = 1, 2, 4

OPS = {
    "rgb2gray": 1, "gauss5": 2, "sobel3": 3, "gradmag": 4, "products": 5,
    "boxsum5": 6, "harris": 7, "threshold": 8, "nms3": 9, "framediff": 10,
    "stencil": 11, "box": 12, "point": 13, "iir": 14,
}
POINT_KINDS = {"affine": 0, "abs": 1, "square": 2, "sqrtabs": 3, "clamp": 4}
OP_NAMES = {v: k for k, v in OPS.items()}

HARRIS_CHAIN = ["gauss5", "sobel3", "products", "boxsum5", "harris", "threshold", "nms3", "framediff"]
RGB_HARRIS_CHAIN = ["rgb2gray"] + HARRIS_CHAIN
GRAD_CHAIN = ["gauss5", "sobel3", "gradmag"]


class FzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fz error {code}: {msg}")
        self.code = code


class fz_stage(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("rx", ctypes.c_int32), ("ry", ctypes.c_int32), ("rt", ctypes.c_int32),
                ("in_ch", ctypes.c_int32), ("out_ch", ctypes.c_int32), ("in_dtype", ctypes.c_int32),
                ("out_dtype", ctypes.c_int32), ("dep", ctypes.c_int32), ("param", ctypes.c_float * 4),
                ("weights", ctypes.POINTER(ctypes.c_float))]


class fz_point(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint32), ("y", ctypes.c_uint32), ("x", ctypes.c_uint32), ("response", ctypes.c_float)]


class fz_plan_opts(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("frames", ctypes.c_int32),
                ("lds_budget_bytes", ctypes.c_int32), ("partition", ctypes.c_int32), ("n_cuts", ctypes.c_int32),
                ("cuts", ctypes.POINTER(ctypes.c_int32)), ("cost_model", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("frames_per_block", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("cost_weights", ctypes.POINTER(ctypes.c_float)),
                ("cost_n_features", ctypes.c_int32)]


class fz_segment_info(ctypes.Structure):
    _fields_ = [("first", ctypes.c_int32), ("last", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("frames_per_block", ctypes.c_int32), ("halo", ctypes.c_int32),
                ("halo_t", ctypes.c_int32), ("lds_bytes", ctypes.c_int32), ("streaming", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("bytes_per_px", ctypes.c_double), ("cost", ctypes.c_double)]


class fz_track_opts(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("r", ctypes.c_double), ("gate", ctypes.c_double), ("v0", ctypes.c_double),
                ("max_miss", ctypes.c_int32), ("max_tracks", ctypes.c_int32)]


class fz_track(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint32), ("id", ctypes.c_uint32), ("status", ctypes.c_int32), ("pad", ctypes.c_uint32),
                ("x", ctypes.c_double), ("y", ctypes.c_double), ("vx", ctypes.c_double), ("vy", ctypes.c_double)]


class fz_clip(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("frames", ctypes.c_int32), ("d_points", ctypes.c_void_p),
                ("d_point_count", ctypes.c_void_p), ("point_capacity", ctypes.c_uint32)]


_lib = None

# (name, restype, argtypes) of every symbol include/fz.h declares
SIGNATURES = [
    ("fz_stage_describe", ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(fz_stage)]),
    ("fz_plan_chain", ctypes.c_int32, [ctypes.POINTER(fz_stage), ctypes.c_int32, ctypes.POINTER(fz_plan_opts),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    ("fz_plan_destroy", None, [ctypes.c_void_p]),
    ("fz_plan_num_segments", ctypes.c_int32, [ctypes.c_void_p]),
    ("fz_plan_segments", ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    ("fz_plan_segment_info", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(fz_segment_info)]),
    ("fz_plan_cost", ctypes.c_double, [ctypes.c_void_p]),
    ("fz_plan_set_segment_config", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int32, ctypes.c_int32]),
    ("fz_plan_group_cost", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double)]),
    ("fz_partition_min", ctypes.c_int32, [ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_double)]),
    ("fz_workspace_bytes", ctypes.c_size_t, [ctypes.c_void_p]),
    ("fz_measure_workspace_bytes", ctypes.c_size_t, [ctypes.c_void_p]),
    ("fz_plan_measure", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_int32, ctypes.c_void_p]),
    ("fz_run_chain", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]),
    ("fz_run_chain_static", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]),
    ("fz_batch_workspace_bytes", ctypes.c_size_t, [ctypes.c_void_p, ctypes.POINTER(fz_clip), ctypes.c_int32]),
    ("fz_run_batch", ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(fz_clip), ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p]),
    ("fz_cost_n_features", ctypes.c_int32, []),
    ("fz_plan_segment_features", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                                  ctypes.c_int32]),
    ("fz_mlp_param_count", ctypes.c_int32, [ctypes.c_int32]),
    ("fz_mlp_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    ("fz_mlp_forward", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    ("fz_mlp_loss_grad", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    ("fz_mlp_adam_step", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, ctypes.c_void_p]),
    ("fz_box_eq6", ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("fz_track_default_opts", ctypes.c_int32, [ctypes.POINTER(fz_track_opts)]),
    ("fz_track_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(fz_track_opts)]),
    ("fz_track_points", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32,
                                         ctypes.POINTER(fz_track_opts), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("fz_last_error", ctypes.c_char_p, []),
    ("fz_version", ctypes.c_char_p, []),
]


def _torch_runtime_first():
    """Initialise torch's GPU runtime before the library is loaded.

    The library and PyTorch's ROCm build may each bring a HIP runtime into the
    process; the device buffers and streams the binding passes come from
    torch's.  Loading the library first and initialising torch afterwards has
    left the library's runtime without a device, so torch goes first (a no-op
    without a GPU or without torch)."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                              f"python paper_1509_04394_amd/build.py")
        _torch_runtime_first()
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != FZ_OK:
        raise FzError(rc, fz_last_error())


def fz_last_error() -> str:
    return lib().fz_last_error().decode()


def fz_version() -> str:
    return lib().fz_version().decode()


def fz_stage_describe(op) -> fz_stage:
    s = fz_stage()
    _check(lib().fz_stage_describe(OPS[op] if isinstance(op, str) else int(op), ctypes.byref(s)))
    return s


def fz_plan_chain(stages, opts: fz_plan_opts) -> ctypes.c_void_p:
    arr = (fz_stage * len(stages))(*stages)
    h = ctypes.c_void_p()
    _check(lib().fz_plan_chain(arr, len(stages), ctypes.byref(opts), ctypes.byref(h)))
    return h


def fz_plan_destroy(plan):
    lib().fz_plan_destroy(plan)


def fz_plan_num_segments(plan) -> int:
    return lib().fz_plan_num_segments(plan)


def fz_plan_segments(plan) -> list[int]:
    n = fz_plan_num_segments(plan)
    buf = (ctypes.c_int32 * max(n, 1))()
    _check(lib().fz_plan_segments(plan, buf, n))
    return list(buf[:n])


def fz_plan_segment_info(plan, i) -> fz_segment_info:
    s = fz_segment_info()
    _check(lib().fz_plan_segment_info(plan, i, ctypes.byref(s)))
    return s


def fz_plan_set_segment_config(plan, i, engine, tile_w=0, tile_h=0, frames_per_block=0):
    eng = ENGINES[engine] if isinstance(engine, str) else int(engine)
    _check(lib().fz_plan_set_segment_config(plan, i, eng, tile_w, tile_h, frames_per_block))


def fz_plan_cost(plan) -> float:
    return lib().fz_plan_cost(plan)


def fz_plan_group_cost(plan, a, b) -> float:
    c = ctypes.c_double()
    _check(lib().fz_plan_group_cost(plan, a, b, ctypes.byref(c)))
    return c.value


def fz_partition_min(cost) -> tuple[float, list[int]]:
    """cost: n x n nested list / array (inf = not allowed). Returns (total, seg_last)."""
    n = len(cost)
    flat = (ctypes.c_double * (n * n))()
    for a in range(n):
        for b in range(n):
            v = cost[a][b] if b >= a else math.inf
            flat[a * n + b] = math.inf if v is None else float(v)
    sl = (ctypes.c_int32 * n)()
    ns = ctypes.c_int32()
    tot = ctypes.c_double()
    _check(lib().fz_partition_min(flat, n, sl, ctypes.byref(ns), ctypes.byref(tot)))
    return tot.value, list(sl[:ns.value])


def fz_workspace_bytes(plan) -> int:
    return int(lib().fz_workspace_bytes(plan))


def fz_measure_workspace_bytes(plan) -> int:
    return int(lib().fz_measure_workspace_bytes(plan))


def fz_plan_measure(plan, d_in, d_workspace, ws_bytes, reps, stream):
    _check(lib().fz_plan_measure(plan, d_in, d_workspace, ws_bytes, reps, stream))


def fz_run_chain(plan, d_in, d_out, d_points, d_point_count, point_capacity, d_workspace, ws_bytes, stream):
    _check(lib().fz_run_chain(plan, d_in, d_out, d_points, d_point_count, point_capacity, d_workspace, ws_bytes,
                              stream))


FZ_STATIC_WORKSPACE_BYTES = 64 << 20


def fz_run_chain_static(plan, d_in, d_out, d_points, d_point_count, point_capacity, stream):
    _check(lib().fz_run_chain_static(plan, d_in, d_out, d_points, d_point_count, point_capacity, stream))


def fz_box_eq6(beta, dx, dt):
    """Sec. VI-E, Eq. 6: (x, t) of the box x*x*t of volume beta whose input
    box (x + 2 dx)^2 (t + dt) is least."""
    x, t = ctypes.c_double(), ctypes.c_double()
    _check(lib().fz_box_eq6(float(beta), float(dx), float(dt), ctypes.byref(x), ctypes.byref(t)))
    return x.value, t.value


def fz_track_points(d_points, d_point_count, point_capacity, frames, opts, d_tracks, d_track_count,
                    track_capacity, d_workspace, ws_bytes, stream):
    _check(lib().fz_track_points(d_points, d_point_count, point_capacity, int(frames), ctypes.byref(opts), d_tracks,
                                 d_track_count, track_capacity, d_workspace, ws_bytes, stream))


def fz_track_workspace_bytes(frames, point_capacity, opts) -> int:
    return int(lib().fz_track_workspace_bytes(int(frames), int(point_capacity), ctypes.byref(opts)))


def track_opts(**kw):
    """fz_track_opts with the library's defaults, fields overridden by kw."""
    o = fz_track_opts()
    _check(lib().fz_track_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def track_points(points, count, frames, opts=None, capacity=None, stream=None):
    """Kalman tracking (fz_track_points) of a point buffer (device tensors as
    Plan.run returns them: points (cap, 4) int32, count (>= 1) int32) over a
    clip of `frames` frames.  Returns (records numpy structured rows (t, id,
    status, x, y, vx, vy), flags).  Synchronises."""
    import torch
    o = opts or track_opts()
    check_points(points, count, points.device if points is not None else None)
    dev = count.device
    cap_in = points.shape[0] if points is not None else 0
    if capacity is None:
        capacity = max(1024, 4 * cap_in * (o.max_miss + 2))
    out = torch.empty((max(capacity, 1), 12), dtype=torch.int32, device=dev)  # 48-byte records
    tc = torch.zeros((2,), dtype=torch.int32, device=dev)
    need = int(lib().fz_track_workspace_bytes(int(frames), cap_in, ctypes.byref(o)))
    ws = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    _check(lib().fz_track_points(points.data_ptr() if points is not None else None, count.data_ptr(), cap_in,
                                 int(frames), ctypes.byref(o), out.data_ptr(), tc.data_ptr(), capacity,
                                 ws.data_ptr(), ws.numel(), stream))
    torch.cuda.synchronize(dev)
    n, flags = int(tc[0].item()), int(tc[1].item())
    if n > capacity:
        raise RuntimeError(f"track buffer overflow: {n} records, capacity {capacity}")
    raw = out[:n].cpu().numpy()
    dt = np.dtype([("t", "<u4"), ("id", "<u4"), ("status", "<i4"), ("pad", "<u4"), ("x", "<f8"), ("y", "<f8"),
                   ("vx", "<f8"), ("vy", "<f8")])
    return raw.view(dt).reshape(-1), flags


def fz_batch_workspace_bytes(plan, clips) -> int:
    arr = (fz_clip * len(clips))(*clips)
    return int(lib().fz_batch_workspace_bytes(plan, arr, len(clips)))


def fz_run_batch(plan, clips, d_workspace, ws_bytes, stream):
    arr = (fz_clip * len(clips))(*clips)
    _check(lib().fz_run_batch(plan, arr, len(clips), d_workspace, ws_bytes, stream))


def fz_cost_n_features() -> int:
    return int(lib().fz_cost_n_features())


def fz_plan_segment_features(plan, i):
    n = fz_cost_n_features()
    buf = (ctypes.c_float * n)()
    r = lib().fz_plan_segment_features(plan, i, buf, n)
    if r < 0:
        raise FzError(FZ_E_INVALID, fz_last_error())
    return list(buf[:r])


def fz_mlp_param_count(n_features) -> int:
    return int(lib().fz_mlp_param_count(n_features))


def fz_mlp_workspace_bytes(n_features, n) -> int:
    return int(lib().fz_mlp_workspace_bytes(n_features, n))


def fz_mlp_forward(d_params, n_features, d_x, n, d_y, stream):
    _check(lib().fz_mlp_forward(d_params, n_features, d_x, n, d_y, stream))


def fz_mlp_loss_grad(d_params, n_features, d_x, d_target, n, d_grad, d_loss, d_ws, ws_bytes, stream):
    _check(lib().fz_mlp_loss_grad(d_params, n_features, d_x, d_target, n, d_grad, d_loss, d_ws, ws_bytes, stream))


def fz_mlp_adam_step(d_params, d_grad, d_m, d_v, n_params, step, lr, beta1, beta2, eps, stream):
    _check(lib().fz_mlp_adam_step(d_params, d_grad, d_m, d_v, n_params, step, lr, beta1, beta2, eps, stream))


# ---------------------------------------------------------------- convenience wrapper
def make_opts(W, H, T, partition="optimal", lds_budget=0, tile=None, frames_per_block=0, cost_model="analytic",
              engine="auto", band_h=0, cost_weights=None):
    o = fz_plan_opts()
    o.width, o.height, o.frames = int(W), int(H), int(T)
    o.lds_budget_bytes = int(lds_budget)
    o._cuts = None
    if partition == "optimal":
        o.partition = FZ_PART_OPTIMAL
    elif partition == "unfused":
        o.partition = FZ_PART_UNFUSED
    else:
        cuts = list(partition)
        o.partition = FZ_PART_EXPLICIT
        o._cuts = (ctypes.c_int32 * max(len(cuts), 1))(*cuts)
        o.cuts = ctypes.cast(o._cuts, ctypes.POINTER(ctypes.c_int32))
        o.n_cuts = len(cuts)
    o.cost_model = {"analytic": FZ_COST_ANALYTIC, "learned": FZ_COST_LEARNED, "measured": FZ_COST_MEASURED}[cost_model]
    if tile is not None:
        o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.frames_per_block = int(frames_per_block)
    o.engine = ENGINES[engine]
    if cost_weights is not None:
        o._w = (ctypes.c_float * len(cost_weights))(*[float(v) for v in cost_weights])
        o.cost_weights = ctypes.cast(o._w, ctypes.POINTER(ctypes.c_float))
        o.cost_n_features = fz_cost_n_features()
    if band_h:
        o.tile_h = int(band_h)  # row engine: rows per band (tile_w stays 0)
    return o


def generic_stages(spec, in_dtype="u8"):
    """fz_stage descriptors for a generic chain given as tuples
    ("stencil", rx, ry, w[2ry+1][2rx+1]) (or w[rt+1][2ry+1][2rx+1]: a stencil
    that also reads the rt frames before t, w[tau] on frame t - tau), ("box",
    rx, ry), ("point", kind, a, b) (kind a name of POINT_KINDS) or ("iir", a).  The first stage reads `in_dtype` ("u8" or
    "f32").  Returns (stages, keep): `keep` holds the weight arrays the
    descriptors point to until the plan has copied them."""
    stages, keep = [], []
    for i, st in enumerate(spec):
        s = fz_stage_describe(st[0])
        if st[0] == "point":
            s.param[0] = float(POINT_KINDS[st[1]])
            s.param[1] = float(st[2]) if len(st) > 2 else 0.0
            s.param[2] = float(st[3]) if len(st) > 3 else 0.0
        elif st[0] == "iir":
            s.param[0] = float(st[1])
        else:
            s.rx, s.ry = int(st[1]), int(st[2])
            if st[0] == "stencil":
                w = np.asarray(st[3], np.float64)
                if w.ndim not in (2, 3) or w.shape[-2:] != (2 * s.ry + 1, 2 * s.rx + 1):
                    raise ValueError(f"stage {i}: stencil weights must have shape ([rt+1,] {2 * s.ry + 1}, "
                                     f"{2 * s.rx + 1}), got {w.shape}")
                if w.ndim == 3:  # frames back: w[tau] multiplies frame t - tau
                    s.rt = w.shape[0] - 1
                w = [float(v) for v in w.ravel()]
                arr = (ctypes.c_float * len(w))(*w)
                keep.append(arr)
                s.weights = ctypes.cast(arr, ctypes.POINTER(ctypes.c_float))
        if i == 0 and in_dtype == "u8":
            s.in_dtype = FZ_U8
        stages.append(s)
    return stages, keep


class Plan:
    """A planned chain for videos of W x H x T.

    ops: op names of the fixed chains, or generic stage tuples (see
    generic_stages; `in_dtype` then gives the input type).
    partition: "optimal" (planner), "unfused" (one kernel per stage) or a list
    of cut positions (last stage index of every group but the final).
    params: optional dict op name -> param[0] (sigma, k or threshold).
    """

    def __init__(self, ops, W, H, T, partition="optimal", lds_budget=0, tile=None, frames_per_block=0,
                 params=None, deps=None, engine="auto", band_h=0, cost_weights=None, in_dtype="u8"):
        self.ops = list(ops)
        self.W, self.H, self.T = int(W), int(H), int(T)
        self.generic = bool(self.ops) and isinstance(self.ops[0], tuple)
        keep = None
        if self.generic:
            stages, keep = generic_stages(self.ops, in_dtype)
            for i, s in enumerate(stages):
                if deps and i in deps:
                    s.dep = int(deps[i])
        else:
            stages = []
            for i, op in enumerate(self.ops):
                s = fz_stage_describe(op)
                if params and op in params:
                    s.param[0] = float(params[op])
                if deps and i in deps:
                    s.dep = int(deps[i])
                stages.append(s)
        self.stages = stages
        self.opts = make_opts(W, H, T, partition, lds_budget, tile, frames_per_block,
                              cost_model="learned" if cost_weights is not None else "analytic",
                              engine=engine, band_h=band_h, cost_weights=cost_weights)
        self.handle = fz_plan_chain(stages, self.opts)
        del keep  # the plan holds its own copy of the weights
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.fz_plan_destroy(h)
            self.handle = None

    # introspection
    @property
    def segments(self):
        return fz_plan_segments(self.handle)

    def segment_info(self):
        return [fz_plan_segment_info(self.handle, i) for i in range(fz_plan_num_segments(self.handle))]

    @property
    def cost(self):
        return fz_plan_cost(self.handle)

    def group_cost(self, a, b):
        return fz_plan_group_cost(self.handle, a, b)

    @property
    def workspace_bytes(self):
        return fz_workspace_bytes(self.handle)

    # shapes
    def input_shape(self):
        s = self.stages[0]
        if s.op == OPS["rgb2gray"]:
            return (self.T, self.H, self.W, 3)
        if s.in_dtype == FZ_U8:
            return (self.T, self.H, self.W)
        return (s.in_ch, self.T, self.H, self.W)

    def output_shape(self):
        s = self.stages[-1]
        if s.out_dtype == FZ_U8:
            return (self.T, self.H, self.W)
        return (s.out_ch, self.T, self.H, self.W)

    def output_dtype(self):
        import torch
        return torch.uint8 if self.stages[-1].out_dtype == FZ_U8 else torch.float32

    def has_points(self):
        return any(s.op == OPS["nms3"] for s in self.stages)

    def measure(self, x, reps=3, stream=None):
        """Replace the prices by measured microseconds on input `x` (a device
        tensor of input_shape()) and re-plan (fz_plan_measure)."""
        import torch
        if tuple(x.shape) != self.input_shape() or not x.is_cuda or not x.is_contiguous():
            raise ValueError("input must be a contiguous CUDA tensor of the plan's input shape")
        ws = torch.empty((fz_measure_workspace_bytes(self.handle),), dtype=torch.uint8, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        fz_plan_measure(self.handle, x.data_ptr(), ws.data_ptr(), ws.numel(), int(reps), stream)
        del ws

    def set_segment_config(self, i, engine="tile", tile=(0, 0), frames_per_block=0):
        fz_plan_set_segment_config(self.handle, i, engine, tile[0], tile[1], frames_per_block)

    def alloc(self, device="cuda", point_capacity=1 << 20):
        """Allocate (out, points, count, workspace) tensors for a run."""
        import torch
        out = torch.empty(self.output_shape(), dtype=self.output_dtype(), device=device)
        pts = cnt = None
        if self.has_points() and point_capacity > 0:
            pts = torch.empty((point_capacity, 4), dtype=torch.int32, device=device)
            cnt = torch.zeros((1,), dtype=torch.int32, device=device)
        ws = torch.empty((max(self.workspace_bytes, 1),), dtype=torch.uint8, device=device)
        return out, pts, cnt, ws

    def input_dtype(self):
        import torch
        return torch.uint8 if self.stages[0].in_dtype == FZ_U8 else torch.float32

    def run(self, x, out=None, points=None, count=None, workspace=None, stream=None):
        """Run on device tensors (asynchronous on the current torch stream).
        Every buffer is checked for shape, type, device and contiguity before
        the C call: a wrong buffer would otherwise be read or written out of
        bounds on the device."""
        import torch
        check_tensor(x, self.input_shape(), self.input_dtype(), "input")
        if out is None:
            out, p2, c2, ws2 = self.alloc(x.device)
            points = points if points is not None else p2
            count = count if count is not None else c2
            workspace = workspace if workspace is not None else ws2
        if workspace is None:
            workspace = torch.empty((max(self.workspace_bytes, 1),), dtype=torch.uint8, device=x.device)
        check_tensor(out, self.output_shape(), self.output_dtype(), "output", x.device)
        check_points(points, count, x.device)
        check_tensor(workspace, None, torch.uint8, "workspace", x.device)
        if workspace.numel() < self.workspace_bytes:
            raise ValueError(f"workspace has {workspace.numel()} bytes, the plan needs {self.workspace_bytes}")
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        cap = points.shape[0] if points is not None else 0
        fz_run_chain(self.handle, x.data_ptr(), out.data_ptr(),
                     points.data_ptr() if points is not None else None,
                     count.data_ptr() if count is not None else None, cap,
                     workspace.data_ptr(), workspace.numel(), stream)
        return out, points, count


    def run_static(self, x, out=None, points=None, count=None, stream=None):
        """fz_run_chain_static: the same run with the library's own fixed
        workspace (no workspace tensor).  Buffers are checked as in run()."""
        import torch
        check_tensor(x, self.input_shape(), self.input_dtype(), "input")
        if out is None:
            out = torch.empty(self.output_shape(), dtype=self.output_dtype(), device=x.device)
        check_tensor(out, self.output_shape(), self.output_dtype(), "output", x.device)
        check_points(points, count, x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        cap = points.shape[0] if points is not None else 0
        fz_run_chain_static(self.handle, x.data_ptr(), out.data_ptr(),
                            points.data_ptr() if points is not None else None,
                            count.data_ptr() if count is not None else None, cap, stream)
        return out, points, count

def check_tensor(t, shape, dtype, what, device=None):
    """A contiguous CUDA tensor of the given dtype (and shape, and device)."""
    if t is None or not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} shape {tuple(t.shape)} != {tuple(shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{what} is on {t.device}, the input on {device}")


def check_points(points, count, device=None):
    """Feature-point buffer: (capacity, 4) int32 records {t, y, x, response};
    count: at least one int32 (the library writes one uint32)."""
    import torch
    if points is not None:
        check_tensor(points, None, torch.int32, "points", device)
        if points.dim() != 2 or points.shape[1] != 4:
            raise ValueError(f"points must be (capacity, 4) int32, got shape {tuple(points.shape)}")
    if count is not None:
        check_tensor(count, None, torch.int32, "count", device)
        if count.numel() < 1:
            raise ValueError("count must hold at least one int32")
    if points is not None and count is None:
        raise ValueError("a point buffer needs a count")


def clip_shapes(ops_plan, W, H, T):
    """(input shape, output shape) of a clip of W x H x T for a plan's chain."""
    s0, s1 = ops_plan.stages[0], ops_plan.stages[-1]
    if s0.op == OPS["rgb2gray"]:
        ins = (T, H, W, 3)
    elif s0.in_dtype == FZ_U8:
        ins = (T, H, W)
    else:
        ins = (s0.in_ch, T, H, W)
    outs = (T, H, W) if s1.out_dtype == FZ_U8 else (s1.out_ch, T, H, W)
    return ins, outs


def make_clip(x, out, points=None, count=None, width=None, height=None, frames=None, plan=None):
    """fz_clip for device tensors x (input) and out (output); sizes from out's shape
    unless given.  With `plan`, x and out are checked against the clip shapes of
    the plan's chain; either way both must hold the clip's W*H*T pixels."""
    import torch
    c = fz_clip()
    shp = out.shape[-3:]
    c.frames, c.height, c.width = (int(frames or shp[0]), int(height or shp[1]), int(width or shp[2]))
    if plan is not None:
        ins, outs = clip_shapes(plan, c.width, c.height, c.frames)
        check_tensor(x, ins, plan.input_dtype(), "clip input")
        check_tensor(out, outs, plan.output_dtype(), "clip output", x.device)
    else:
        npx = c.width * c.height * c.frames
        for t, what in ((x, "clip input"), (out, "clip output")):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{what} must be a contiguous CUDA tensor")
            if t.dtype not in (torch.uint8, torch.float32) or t.numel() % npx != 0 or t.numel() == 0:
                raise ValueError(f"{what} ({tuple(t.shape)}, {t.dtype}) does not hold {npx} pixels")
    check_points(points, count, x.device)
    c.d_in = x.data_ptr()
    c.d_out = out.data_ptr()
    c.d_points = points.data_ptr() if points is not None else None
    c.d_point_count = count.data_ptr() if count is not None else None
    c.point_capacity = int(points.shape[0]) if points is not None else 0
    return c


def run_batch(plan: "Plan", clips, workspace=None, stream=None):
    """Run `plan` over fz_clip descriptors (device buffers owned by the caller)."""
    import torch
    need = fz_batch_workspace_bytes(plan.handle, clips)
    if workspace is None:
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    fz_run_batch(plan.handle, clips, workspace.data_ptr(), workspace.numel(), stream)
    return workspace


def points_to_numpy(points, count):
    """Device point buffer -> numpy array rows (t, y, x, response), count-limited."""
    import numpy as np
    n = int(count.item())
    cap = points.shape[0]
    if n > cap:
        raise RuntimeError(f"point buffer overflow: {n} > {cap}")
    raw = points[:n].cpu().numpy()
    out = np.empty((n, 4), np.float64)
    out[:, :3] = raw[:, :3].view(np.uint32)
    out[:, 3] = raw[:, 3].view(np.float32)
    return out
