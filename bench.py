"""Benchmark of the fused video-kernel chain on one MI355X.

Default workload: 800x600x1000 RGB uint8 video (synthetic, seeded), rgb2gray
followed by the 8-stage Harris chain (Gaussian 5x5, Sobel, structure products,
5x5 window sums, Harris response, threshold, 3x3 suppression, frame
difference), partition chosen by the planner (full fusion).  One step = one
pass of the whole chain over the whole video, input already resident in HBM.

Prints one JSON line: fused throughput in Mpixel/s (`value`), the roofline of
the dominant kernel (its launches timed with HIP events on the stream they run
on, inside the timed region), and beside them, measured in the same process:
the unfused sequence, the paper's "Two Fusion" partition, the input handed
over from host memory, the smaller workloads (192x432 gray, gradient and
Harris chains) fused and unfused, the 32-clip batch (one persistent graph
launch against one launch per clip) and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for roofline fractions
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ, LANES_PER_CU = 256, 2.4, 64  # 4 SIMDs x 16 lanes
VALU_PEAK_GOPS = N_CU * LANES_PER_CU * CLOCK_GHZ  # 39,321.6 G lane-ops/s (non-packed)

WORKLOADS = {
    "rgb800": dict(W=800, H=600, T=1000, rgb=True, seed=3, chain="rgb_harris",
                   desc="800x600x1000 RGB u8, rgb2gray + 8-stage Harris chain"),
    "harris192": dict(W=192, H=432, T=600, rgb=False, seed=2, chain="harris",
                      desc="192x432x600 gray u8, 8-stage Harris chain"),
    "grad192": dict(W=192, H=432, T=64, rgb=False, seed=1, chain="grad",
                    desc="192x432x64 gray u8, Gaussian -> Sobel -> magnitude"),
    "generic800": dict(W=800, H=600, T=64, rgb=False, seed=6, chain="generic3",
                       desc="800x600x64 gray u8, plan-time generic chain: 3x3 stencil -> |x| -> 3x3 window sum"),
    "paper5_800": dict(W=800, H=600, T=1000, rgb=False, seed=7, chain="paper5",
                       desc="800x600x1000 gray u8, the paper's five-kernel chain with generic stages: IIR (a = 0.3) "
                            "-> 5x5 Gaussian -> 3x3 horizontal Sobel -> |x| -> clamp [0, 200]"),
    "spatio800": dict(W=800, H=600, T=1000, rgb=False, seed=8, chain="spatio",
                      desc="800x600x1000 gray u8, stencils that look back: affine -> 3x3 over 3 frames -> 3x3 "
                           "window sum -> 5x3 over 2 frames -> sqrt|x|"),
    "batch32": dict(W=800, H=600, T=1000, rgb=False, seed=4, chain="harris", clips=32,
                    desc="32 gray u8 clips, frame sizes drawn from 192x432 / 320x240 / 640x480 / 800x600, "
                         "50-1000 frames, 8-stage Harris chain, one persistent graph launch"),
}
METRIC = "Mpixel/s fused vs unfused and HBM GB/s (% of peak), 800×600×1000 chain"

# Algorithmic VALU operations per output pixel, two counts:
#  * MIN_OPS: the least work of each stage (separable passes, every
#    intermediate formed once, 5x5 window sums as running sums);
#  * KERNEL_OPS: the least work in the summation order every engine of the
#    library keeps so that all partitions give the same bits -- the u8 -> f32
#    conversion counted in the Gaussian (+1), and each 5-wide window sum as
#    ((a+b)+(c+d))+e with the pair sums shared by neighbouring windows (3 + 3
#    additions per channel instead of a running sum's 2 + 2: +6).
MIN_OPS = {"rgb2gray": 9, "gauss5": 10, "sobel3": 6, "gradmag": 3, "products": 3, "boxsum5": 12,
           "harris": 5, "threshold": 2, "nms3": 7, "framediff": 2}
KERNEL_OPS = dict(MIN_OPS, gauss5=11, boxsum5=18)

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes, scaled by the plain-copy calibration (profiles/rowfuse_rgb800_counters.md).
# Valid only for the kernel sources and the launch geometry (columns per strip,
# band rows, frames per work item) they were taken with: the key holds both.
COUNTER_TRAFFIC = {
    ("rgb800", "1317c82aa13af6db", (128, 75, 2)): {"fetch_bytes": 2.029e9, "write_bytes": 0.660e9,
                                                   "source": "profiles/rowfuse_rgb800_counters.md"},
}
KERNEL_SOURCES = ["rowfuse.h", "stage_math.h"]
DRIVER_TIMEOUT_S = 600


def kernel_source_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_1509_04394_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(d, f), "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def chain_ops(name):
    from paper_1509_04394_amd import fz
    if name == "generic3":  # stages given at plan time (weights: the 3x3 binomial, normalised)
        w3 = (np.outer([1, 2, 1], [1, 2, 1]) / 16.0).astype(np.float32)
        return [("stencil", 1, 1, w3), ("point", "abs", 0.0, 0.0), ("box", 1, 1)]
    if name == "paper5":  # IIR -> Gaussian -> gradient -> magnitude -> clamp (Table II's kernels K2..K5)
        g = np.exp(-np.arange(-2, 3) ** 2 / 2.0)
        g5 = (np.outer(g, g) / np.outer(g, g).sum()).astype(np.float32)
        sx = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], np.float32)
        return [("iir", float(np.float32(0.3))), ("stencil", 2, 2, g5), ("stencil", 1, 1, sx),
                ("point", "abs", 0.0, 0.0), ("point", "clamp", 0.0, 200.0)]
    if name == "spatio":  # stencils over several frames (Table I, spatio-temporal)
        w33 = (np.arange(27, dtype=np.float32).reshape(3, 3, 3) % 5 + 1.0) / 60.0
        w253 = ((np.arange(30, dtype=np.float32).reshape(2, 3, 5) % 7) - 3.0) / 40.0
        return [("point", "affine", 0.5, 1.0), ("stencil", 1, 1, w33), ("box", 1, 1), ("stencil", 2, 1, w253),
                ("point", "sqrtabs", 0.0, 0.0)]
    return {"rgb_harris": fz.RGB_HARRIS_CHAIN, "harris": fz.HARRIS_CHAIN, "grad": fz.GRAD_CHAIN}[name]


def ops_per_px(ops, table=None):
    """Algorithmic VALU operations per output pixel of a chain (KERNEL_OPS by
    default).  Generic stages: one multiply-add per stencil tap, one addition
    per window element, one operation per point stage (two for a clamp)."""
    table = table or KERNEL_OPS

    def generic(st):
        if st[0] == "point":
            return 2 if st[1] == "clamp" else 1
        if st[0] == "iir":
            return 2
        frames = np.asarray(st[3]).shape[0] if st[0] == "stencil" and np.asarray(st[3]).ndim == 3 else 1
        return (2 * st[1] + 1) * (2 * st[2] + 1) * frames
    return sum(generic(o) if isinstance(o, tuple) else table[o] for o in ops)


def hbm_bytes_per_px(plan, first, last):
    """Algorithmic bytes per pixel of the group first..last of a plan: its input
    read once and its output written once (the frame difference's temporal
    halo re-read is not counted)."""
    a, b = plan.stages[first], plan.stages[last]
    size = lambda dt: 4 if dt == 2 else 1
    return a.in_ch * size(a.in_dtype) + b.out_ch * size(b.out_dtype)


def time_plan(plan, x, bufs, steps, warmup, stream):
    """Time `steps` runs back to back after `warmup` untimed runs.  Each run is
    bracketed by its own pair of HIP events on `stream`; the events of one run
    follow the previous run's with no synchronisation between them, so the
    region from the first to the last event is the back-to-back time.
    Returns (ms per step over the region, mean per-run event time, per-run times)."""
    import torch
    out, pts, cnt, ws = bufs
    for _ in range(warmup):
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
        b.record(stream)
    torch.cuda.synchronize()
    times = [a.elapsed_time(b) for a, b in evs]
    region = evs[0][0].elapsed_time(evs[-1][1]) / steps
    return float(region), float(np.mean(times)), times


def copy_ceiling_gbs(dev, nbytes=1 << 30, reps=5):
    """Same-run device-to-device copy rate: (bytes read + bytes written) / time, GB/s."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def pcie_inclusive(plan, x, bufs, stream, reps=3):
    """End-to-end time of one pass including the host-to-device copy of the
    input from pinned host memory (ms), and the copy alone (ms)."""
    import torch
    host = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
    host.copy_(x)
    out, pts, cnt, ws = bufs
    torch.cuda.synchronize()
    tot, cp = [], []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        m = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        x.copy_(host, non_blocking=True)
        m.record(stream)
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
        b.record(stream)
        torch.cuda.synchronize()
        tot.append(a.elapsed_time(b))
        cp.append(a.elapsed_time(m))
    del host
    return float(np.median(tot)), float(np.median(cp))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, ops, budget_s=15.0, one_thread_s=3.0):
    """The oracle (FP64, unfused) on a bounded sample of the same workload:
    all host threads, then one thread on a smaller sample.  The uint8 ->
    float64 conversion of the input happens before the timed call."""
    import oracle
    from paper_1509_04394_amd import synth
    oracle.build(force=False)
    cores = os.cpu_count() or 1
    W, H = wl["W"], wl["H"]
    generic = any(isinstance(o, tuple) for o in ops)

    def sample(frames):
        vol = synth.video(W, H, frames, seed=wl["seed"], rgb=wl["rgb"])
        return np.ascontiguousarray(vol, dtype=np.float64) if generic else oracle.to_planes(ops, vol)

    def run(inp, k):
        t = time.perf_counter()
        if generic:
            oracle.gchain(ops, inp, nthreads=k)
        else:
            oracle.chain_planes(ops, inp, nthreads=k)
        return time.perf_counter() - t

    n = 8
    dt = run(sample(n), cores)
    frames = int(min(wl["T"], max(n, n * budget_s / max(dt, 1e-3))))
    frames = max(cores, frames - frames % cores) if frames >= cores else frames
    inp = sample(frames)
    dt = run(inp, min(cores, frames))
    del inp
    px = W * H * frames
    rec = {"value": px / dt / 1e6, "unit": "Mpixel/s", "cores": min(cores, frames), "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"frames 0-{frames - 1} of the {W}x{H}x{wl['T']} workload ({px / 1e6:.1f} Mpx), "
                     f"whole chain unfused in FP64, {dt:.1f} s (input converted to FP64 before timing)"}
    n1 = max(1, int(frames * one_thread_s / max(dt * min(cores, frames), 1e-3)))
    n1 = min(n1, frames)
    inp = sample(n1)
    dt1 = run(inp, 1)
    rec["one_thread"] = {"value": W * H * n1 / dt1 / 1e6, "unit": "Mpixel/s", "cores": 1,
                         "sample": f"frames 0-{n1 - 1} ({W * H * n1 / 1e6:.1f} Mpx), {dt1:.1f} s"}
    return rec


def fused_and_unfused(ops, W, H, T, seed, rgb, steps, warmup, dev, stream, hbm=False):
    """Mpixel/s of the planner's partition and of one kernel per stage on
    another workload (whole video resident in HBM).  With `hbm`, each form's
    algorithmic bytes (every group's input once and output once) over its
    time, and the fused plan's groups (engine, tile, frames per work item)."""
    import torch
    from paper_1509_04394_amd import fz, synth
    x = torch.from_numpy(synth.video(W, H, T, seed=seed, rgb=rgb)).to(dev)
    res = {}
    for name, part in (("fused", "optimal"), ("unfused", "unfused")):
        plan = fz.Plan(ops, W, H, T, partition=part)
        bufs = plan.alloc(dev)
        ms, _, _ = time_plan(plan, x, bufs, steps, warmup, stream)
        res[name] = {"ms_per_step": round(ms, 4), "mpx_s": round(W * H * T / (ms * 1e-3) / 1e6, 1),
                     "partition": plan.segments}
        if hbm:
            byts = sum(hbm_bytes_per_px(plan, s.first, s.last) for s in plan.segment_info()) * W * H * T
            gbs = byts / (ms * 1e-3) / 1e9
            res[name].update(algorithmic_GBs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
            if name == "fused":
                eng = {fz.FZ_ENGINE_ROW: "row", fz.FZ_ENGINE_TILE: "tile", fz.FZ_ENGINE_STREAM: "stream",
                       fz.FZ_ENGINE_JIT: "jit"}
                res[name]["groups"] = [[s.first, s.last, eng[s.engine], s.tile_w, s.tile_h, s.frames_per_block]
                                       for s in plan.segment_info()]
        log(f"  {name}: {ms:.3f} ms/step, partition {plan.segments}")
        del bufs
    res["speedup_vs_unfused"] = round(res["unfused"]["ms_per_step"] / res["fused"]["ms_per_step"], 3)
    del x
    torch.cuda.empty_cache()
    return res


def tracking_leg(points, count, T, stream, reps=3, cpu=True):
    """The Kalman tracking stage after the chain (its own launches on the
    chain's point list): ms per pass over the whole clip, records and tracks;
    beside it the oracle tracking the same points on one host thread."""
    import torch
    from paper_1509_04394_amd import fz
    rec, flags = fz.track_points(points, count, T)  # the records (and a warm-up)
    o = fz.track_opts()
    cap = points.shape[0]
    out = torch.empty((max(len(rec), 1), 12), dtype=torch.int32, device=points.device)
    tc = torch.zeros((2,), dtype=torch.int32, device=points.device)
    ws = torch.empty((fz.fz_track_workspace_bytes(T, cap, o),), dtype=torch.uint8, device=points.device)
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fz.fz_track_points(points.data_ptr(), count.data_ptr(), cap, T, o, out.data_ptr(), tc.data_ptr(),
                           out.shape[0], ws.data_ptr(), ws.numel(), stream.cuda_stream)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    del out, ws
    ms = float(np.median(times))
    n = int(count.item())
    res = {"ms_per_pass": round(ms, 3), "points": n, "records": int(len(rec)), "tracks": int(len(set(rec["id"].tolist()))),
           "flags": flags, "points_per_s": round(n / (ms * 1e-3), 1),
           "note": "Table II's Kalman filter on the chain's feature points, kernel-to-kernel after the chain "
                   "(bucketing by frame, then one workgroup of four wavefronts marching the frames); latency-bound, sequential in t"}
    if cpu:
        import oracle
        host = points[:n, :3].cpu().numpy()
        t0 = time.perf_counter()
        oracle.track(host, T)
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"ms_per_pass": round(dt * 1e3, 3), "cores": 1, "kind": "oracle"}
    log(f"tracking: {ms:.3f} ms for {n} points, {len(rec)} records")
    return res


def autotune_leg(ops, W, H, T, x, steps, warmup, dev, stream, planner_ms):
    """The fused plan after the autotuner (every band / frame run around the
    Eq. 6 seed and every tile timed on the input, the fastest kept), timed as
    the headline is, beside the planner-sized headline."""
    from paper_1509_04394_amd import autotune, fz
    plan = fz.Plan(ops, W, H, T)
    stats = {}
    autotune.autotune(plan, x, reps=3, stats=stats)
    bufs = plan.alloc(dev)
    ms, _, _ = time_plan(plan, x, bufs, steps, warmup, stream)
    del bufs
    s = plan.segment_info()
    log(f"autotuned: {ms:.4f} ms/step ({[(g.tile_w, g.tile_h, g.frames_per_block) for g in s]})")
    return {"ms_per_step": round(ms, 4), "mpx_s": round(W * H * T / (ms * 1e-3) / 1e6, 1),
            "groups": [[g.first, g.last, g.engine, g.tile_w, g.tile_h, g.frames_per_block] for g in s],
            "configs_tried": stats.get("tried", 0), "planner_ms_per_step": round(planner_ms, 4),
            "speedup_over_planner": round(planner_ms / ms, 3)}


def engines_leg(key, steps, warmup, dev, stream):
    """A generic workload fused with the interpreted kernels, fused with the
    generated (hipRTC) kernels, and unfused (the planner's partition for the
    fused forms; groups: first, last, tile, frames per work item)."""
    import torch
    from paper_1509_04394_amd import fz, synth
    w = WORKLOADS[key]
    ops = chain_ops(w["chain"])
    W, H, T = w["W"], w["H"], w["T"]
    x = torch.from_numpy(synth.video(W, H, T, seed=w["seed"])).to(dev)
    res = {"workload": w["desc"]}
    for name, kw in (("fused_tile", dict(engine="tile")), ("fused_jit", dict(engine="jit")),
                     ("unfused", dict(partition="unfused"))):
        plan = fz.Plan(ops, W, H, T, **kw)
        bufs = plan.alloc(dev)
        ms, _, _ = time_plan(plan, x, bufs, steps, warmup, stream)
        byts = sum(hbm_bytes_per_px(plan, s.first, s.last) for s in plan.segment_info()) * W * H * T
        res[name] = {"ms_per_step": round(ms, 4), "mpx_s": round(W * H * T / (ms * 1e-3) / 1e6, 1),
                     "partition": plan.segments, "algorithmic_GBs": round(byts / (ms * 1e-3) / 1e9, 1),
                     "groups": [[s.first, s.last, s.tile_w, s.tile_h, s.frames_per_block]
                                for s in plan.segment_info()]}
        log(f"  {key} {name}: {ms:.4f} ms/step")
        del bufs
    res["jit_over_tile"] = round(res["fused_tile"]["ms_per_step"] / res["fused_jit"]["ms_per_step"], 3)
    res["jit_over_unfused"] = round(res["unfused"]["ms_per_step"] / res["fused_jit"]["ms_per_step"], 3)
    del x
    torch.cuda.empty_cache()
    return res


def batch_leg(wl, steps, warmup, dev, stream):
    """32 clips: one persistent launch replayed from a graph against one
    planned run per clip.  Returns the record (Mpixel/s over all clips)."""
    import torch
    from paper_1509_04394_amd import fz, synth
    ops = chain_ops(wl["chain"])
    shapes = synth.batch_shapes(wl["seed"], wl["clips"])
    npx = sum(W * H * T for W, H, T in shapes)
    log(f"generating {len(shapes)} clips, {npx / 1e9:.2f} Gpx")
    items = []
    for i, (W, H, T) in enumerate(shapes):
        x = torch.from_numpy(synth.video(W, H, T, seed=4000 + i)).to(dev)
        plan = fz.Plan(ops, W, H, T)
        out, pts, cnt, ws = plan.alloc(dev, point_capacity=1 << 18)
        items.append((x, out, pts, cnt, ws, plan))
    bplan = fz.Plan(ops, 800, 600, 1000)
    clips = [fz.make_clip(x, out, pts, cnt, plan=bplan) for (x, out, pts, cnt, _, _) in items]
    bws = torch.empty((max(fz.fz_batch_workspace_bytes(bplan.handle, clips), 1),), dtype=torch.uint8, device=dev)

    def batch_step():
        fz.fz_run_batch(bplan.handle, clips, bws.data_ptr(), bws.numel(), stream.cuda_stream)

    def single_step():
        for (x, out, pts, cnt, w, plan) in items:
            plan.run(x, out, pts, cnt, w, stream=stream.cuda_stream)

    res = {}
    for name, fn in [("batch", batch_step), ("per_clip", single_step)]:
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) / steps
        log(f"batch leg {name}: {res[name]:.3f} ms per pass over all clips")
    alg = sum(W * H * T * 2 for W, H, T in shapes)  # 1 B in + 1 B out per pixel
    rec = {"workload": wl["desc"], "clips": len(shapes), "pixels": npx,
           "ms_per_step": round(res["batch"], 4), "mpx_s": round(npx / (res["batch"] * 1e-3) / 1e6, 1),
           "hbm_algorithmic_GBs": round(alg / (res["batch"] * 1e-3) / 1e9, 1),
           "per_clip_launches": {"ms_per_step": round(res["per_clip"], 4),
                                 "mpx_s": round(npx / (res["per_clip"] * 1e-3) / 1e6, 1)},
           "speedup_vs_per_clip": round(res["per_clip"] / res["batch"], 3)}
    del items, clips, bws
    torch.cuda.empty_cache()
    return rec


def run_batch_workload(args, wl):
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    r = batch_leg(wl, args.steps, args.warmup, dev, stream)
    rec = {"metric": "Mpixel/s, batched clips (persistent graph launch)", "value": r["mpx_s"], "unit": "Mpixel/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "clips": r["clips"], "pixels": r["pixels"]},
           "per_clip_launches": r["per_clip_launches"], "hbm_algorithmic_GBs": r["hbm_algorithmic_GBs"]}
    print(json.dumps(rec), flush=True)


def main():
    wall0 = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed runs first (the GPU clock rises over the first ~10 ms of load)")
    ap.add_argument("--workload", default="rgb800", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--engine", default="auto", choices=["auto", "tile", "row", "jit"],
                    help="kernel family for the fused plan's groups (auto: the planner's choice; jit: generated "
                         "kernels for generic groups)")
    ap.add_argument("--autotune", action="store_true",
                    help="measure every band / tile configuration of each fused group first (untimed) and "
                         "keep the fastest")
    ap.add_argument("--no-unfused", action="store_true", help="skip timing the unfused sequence")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (small configs, batch) in the default run")
    ap.add_argument("--fused-only", action="store_true", help="time only the fused plan (for profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (scale for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not supported (the video would be "
              "split along time, each GPU reading one frame before its range)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1509_04394_amd import fz, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    fz.lib()  # fail loudly if the HIP library is missing
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 5}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    if "clips" in wl:
        run_batch_workload(args, wl)
        return
    ops = chain_ops(wl["chain"])
    W, H, T = wl["W"], wl["H"], wl["T"]
    npx = W * H * T
    dev = torch.device("cuda:0")
    log(f"generating {wl['desc']}")
    t = time.perf_counter()
    vol = synth.video(W, H, T, seed=wl["seed"], rgb=wl["rgb"])
    log(f"generated in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(vol).to(dev)
    del vol
    stream = torch.cuda.current_stream(dev)

    fused = fz.Plan(ops, W, H, T, engine=args.engine)
    if args.autotune:
        from paper_1509_04394_amd import autotune
        log("autotuned", autotune.autotune(fused, x, reps=3))
    info = fused.segment_info()
    fb = fused.alloc(dev)
    log("fused plan groups", fused.segments, "tiles", [(s.tile_w, s.tile_h, s.frames_per_block) for s in info])
    f_ms, f_launch, _ = time_plan(fused, x, fb, args.steps, args.warmup, stream)
    nfused = int(fb[2].item()) if fb[2] is not None else 0
    log(f"fused: {f_ms:.4f} ms/step back to back, {f_launch:.4f} ms mean per run between its events, "
        f"{nfused} points")
    extra = {}
    if nfused and not args.fused_only:
        extra["tracking"] = tracking_leg(fb[1], fb[2], T, stream, cpu=not args.no_cpu)
    if not (args.fused_only or args.autotune):
        extra["autotuned"] = autotune_leg(ops, W, H, T, x, args.steps, args.warmup, dev, stream, f_ms)
    if not args.fused_only:
        e2e, h2d = pcie_inclusive(fused, x, fb, stream)
        extra["pcie_inclusive"] = {
            "ms_per_step": round(e2e, 4), "mpx_s": round(npx / (e2e * 1e-3) / 1e6, 1), "h2d_ms": round(h2d, 4),
            "h2d_GBs": round(x.numel() * x.element_size() / (h2d * 1e-3) / 1e9, 1),
            "note": "input copied from pinned host memory inside the timed pass; not the headline value"}
        log(f"with the host-to-device copy: {e2e:.3f} ms/step ({h2d:.3f} ms copy)")
    copy_gbs = None if args.fused_only else copy_ceiling_gbs(dev)
    del fb
    torch.cuda.empty_cache()

    others = {}
    if not (args.no_unfused or args.fused_only):
        for name, part in (("unfused", "unfused"), ("two_fusion", [1])):
            if name == "two_fusion" and ops != fz.RGB_HARRIS_CHAIN:
                continue
            p = fz.Plan(ops, W, H, T, partition=part, engine=args.engine)
            b = p.alloc(dev)
            ms, _, _ = time_plan(p, x, b, max(3, args.steps // 2), 2, stream)
            log(f"{name}: {ms:.3f} ms/step, partition {p.segments}")
            others[name] = {"mpx_s": round(npx / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                            "partition": p.segments, "kernels": len(p.segments),
                            "algorithmic_GBs": round(p.cost / (ms * 1e-3) / 1e9, 1),
                            "hbm_frac": round(p.cost / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if copy_gbs:
                others[name]["hbm_frac_of_copy"] = round(p.cost / (ms * 1e-3) / 1e9 / copy_gbs, 4)
            del b
            torch.cuda.empty_cache()
        if "two_fusion" in others:
            others["two_fusion"]["note"] = ("the paper's Two Fusion (Sec. VII): the best partition whose "
                                            "groups have halos of at most 4 px, a cut after the Gaussian")
    del x
    torch.cuda.empty_cache()

    # roofline of the dominant kernel: the algorithmic work of one launch over
    # its mean duration between the HIP events around each run in the timed region
    dominant = info[0] if len(info) == 1 else max(info, key=lambda s: s.cost)
    sub = ops[dominant.first:dominant.last + 1]
    opx_min = ops_per_px(sub, MIN_OPS)
    opx_kernel = ops_per_px(sub, KERNEL_OPS)
    gops = npx * opx_min / (f_launch * 1e-3) / 1e9
    bpx = hbm_bytes_per_px(fused, dominant.first, dominant.last)
    gbs = npx * bpx / (f_launch * 1e-3) / 1e9
    traffic = None
    ct = COUNTER_TRAFFIC.get((args.workload, kernel_source_hash(),
                              (dominant.tile_w, dominant.tile_h, dominant.frames_per_block)))
    if ct is not None and dominant.engine == fz.FZ_ENGINE_ROW:
        traffic = round((ct["fetch_bytes"] + ct["write_bytes"]) / (f_launch * 1e-3) / 1e9, 1)
    roof = {"bound": "alu", "achieved": round(gops, 1), "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
            "frac": round(gops / VALU_PEAK_GOPS, 4), "traffic": traffic,
            "traffic_unit": "GB/s (counter bytes per launch / launch time)",
            "ops_per_px": opx_min, "ops_per_px_kernel_order": opx_kernel,
            "frac_kernel_order": round(npx * opx_kernel / (f_launch * 1e-3) / 1e9 / VALU_PEAK_GOPS, 4),
            "launch_ms": round(f_launch, 4), "hbm_bytes_per_px": bpx, "hbm_achieved_GBs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if copy_gbs:
        roof["hbm_frac_of_copy"] = round(gbs / copy_gbs, 4)
    rec = {"metric": METRIC, "value": round(npx / (f_ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(f_ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "partition": fused.segments,
                      "tile": [dominant.tile_w, dominant.tile_h, dominant.frames_per_block],
                      "engine": {fz.FZ_ENGINE_ROW: "row", fz.FZ_ENGINE_TILE: "tile",
                                 fz.FZ_ENGINE_STREAM: "stream", fz.FZ_ENGINE_JIT: "jit"}[dominant.engine],
                      "sizing": "autotuned" if args.autotune else "planner",
                      "points_per_step": nfused},
           "roofline": roof}
    if copy_gbs is not None:
        rec["copy_ceiling_GBs"] = round(copy_gbs, 1)
    rec.update(extra)
    if "unfused" in others:
        rec["unfused"] = others["unfused"]
        rec["speedup_vs_unfused"] = round(others["unfused"]["ms_per_step"] / f_ms, 3)
        rec["paper_context"] = "2-3x fused over sequential kernels on Tesla C1060 / K20 / GTX 750 Ti (Abstract)"
    if "two_fusion" in others:
        rec["two_fusion"] = others["two_fusion"]
    if args.workload == "rgb800" and not (args.no_extra or args.fused_only):
        small = {}
        for key in ("grad192", "harris192"):
            w = WORKLOADS[key]
            log(f"workload {key}")
            small[key] = dict(workload=w["desc"], **fused_and_unfused(
                chain_ops(w["chain"]), w["W"], w["H"], w["T"], w["seed"], w["rgb"], args.steps, args.warmup,
                dev, stream))
        for key in ("paper5_800", "spatio800", "generic800"):
            log(f"workload {key}, interpreted and generated kernels")
            steps = args.steps if key == "generic800" else max(3, args.steps // 4)
            small[key] = engines_leg(key, steps, min(args.warmup, 3), dev, stream)
        rec["other_workloads"] = small
        rec["batched"] = batch_leg(WORKLOADS["batch32"], max(3, args.steps // 4), 2, dev, stream)
    if not (args.no_cpu or args.fused_only):
        log("timing the CPU oracle on a sample")
        rec["cpu_baseline"] = cpu_baseline(wl, ops)
    wall = time.perf_counter() - wall0
    rec["bench_wall_s"] = round(wall, 1)
    rec["fits_in_driver_run"] = wall < 0.8 * DRIVER_TIMEOUT_S
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
