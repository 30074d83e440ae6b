"""Benchmark of the fused video-kernel chain on one MI355X.

Default workload: 800x600x1000 RGB uint8 video (synthetic, seeded), rgb2gray
followed by the 8-stage Harris chain (Gaussian 5x5, Sobel, structure products,
5x5 window sums, Harris response, threshold, 3x3 suppression, frame
difference), partition chosen by the planner (full fusion).  One step = one
pass of the whole chain over the whole video, input already resident in HBM.

Prints one JSON line: fused throughput in Mpixel/s (`value`), the unfused
sequence measured in the same process, the roofline of the dominant kernel
(timed with HIP events on the stream it is launched on) and the CPU oracle on a
bounded sample of the same workload.
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
    "batch32": dict(W=800, H=600, T=1000, rgb=False, seed=4, chain="harris", clips=32,
                    desc="32 gray u8 clips, frame sizes drawn from 192x432 / 320x240 / 640x480 / 800x600, "
                         "50-1000 frames, 8-stage Harris chain, one persistent graph launch"),
}
BATCH_SIZES = [(192, 432), (320, 240), (640, 480), (800, 600)]


def batch_shapes(seed, n):
    rng = np.random.default_rng(seed)
    return [(*BATCH_SIZES[int(rng.integers(0, 4))], int(rng.integers(50, 1001))) for _ in range(n)]


def run_batch_workload(args, wl):
    """32 clips: one persistent launch in a replayed graph vs one launch per clip."""
    import torch
    from paper_1509_04394_amd import fz, synth
    dev = torch.device("cuda:0")
    ops = chain_ops(wl["chain"])
    shapes = batch_shapes(wl["seed"], wl["clips"])
    npx = sum(W * H * T for W, H, T in shapes)
    log(f"generating {len(shapes)} clips, {npx / 1e9:.2f} Gpx")
    items = []
    for i, (W, H, T) in enumerate(shapes):
        x = torch.from_numpy(synth.video(W, H, T, seed=4000 + i)).to(dev)
        plan = fz.Plan(ops, W, H, T)
        out, pts, cnt, ws = plan.alloc(dev, point_capacity=1 << 20)
        items.append((x, out, pts, cnt, ws, plan))
    stream = torch.cuda.current_stream(dev)
    bplan = fz.Plan(ops, 800, 600, 1000)
    clips = [fz.make_clip(x, out, pts, cnt) for (x, out, pts, cnt, _, _) in items]
    ws = torch.empty((max(fz.fz_batch_workspace_bytes(bplan.handle, clips), 1),), dtype=torch.uint8, device=dev)

    def batch_step():
        fz.fz_run_batch(bplan.handle, clips, ws.data_ptr(), ws.numel(), stream.cuda_stream)

    def single_step():
        for (x, out, pts, cnt, w, plan) in items:
            plan.run(x, out, pts, cnt, w, stream=stream.cuda_stream)

    res = {}
    for name, fn in [("batch", batch_step), ("per_clip", single_step)]:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) / args.steps
        log(f"{name}: {res[name]:.3f} ms per pass over all clips")
    value = npx / (res["batch"] * 1e-3) / 1e6
    alg = sum(W * H * T * (1 + 1 + 1.0 / 16) for W, H, T in shapes)
    rec = {"metric": "Mpixel/s, batched clips (persistent graph launch)", "value": round(value, 1),
           "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(res["batch"], 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "clips": len(shapes), "pixels": npx,
                      "shapes": [list(s) for s in shapes]},
           "per_clip_launches": {"ms_per_step": round(res["per_clip"], 4),
                                 "mpx_s": round(npx / (res["per_clip"] * 1e-3) / 1e6, 1)},
           "hbm_algorithmic_GBs": round(alg / (res["batch"] * 1e-3) / 1e9, 1)}
    print(json.dumps(rec), flush=True)

METRIC = "Mpixel/s fused vs unfused and HBM GB/s (% of peak), 800×600×1000 chain"

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes, scaled by the plain-copy calibration (profiles/rowfuse_rgb800_counters.md).
# Valid only for the kernel sources and the launch geometry (columns per strip,
# band rows, frames per work item) they were taken with: the key holds both.
COUNTER_TRAFFIC = {
    ("rgb800", "ed9bc057f0e37bfd", (128, 55, 16)): {"fetch_bytes": 2.488e9, "write_bytes": 0.590e9,
                                                    "source": "profiles/rowfuse_rgb800_counters.md"},
}
KERNEL_SOURCES = ["rowfuse.h", "stage_math.h"]


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
    return {"rgb_harris": fz.RGB_HARRIS_CHAIN, "harris": fz.HARRIS_CHAIN, "grad": fz.GRAD_CHAIN}[name]


def ops_per_px(ops):
    """Algorithmic VALU operations per output pixel: separable passes with every
    intermediate formed once (Sobel from one vertical smoothing and one vertical
    difference per pixel; the 5x5 sums from pair sums that neighbouring windows
    share, horizontally and vertically)."""
    table = {"rgb2gray": 9, "gauss5": 11, "sobel3": 6, "gradmag": 3, "products": 3, "boxsum5": 18,
             "harris": 5, "threshold": 2, "nms3": 7, "framediff": 2}

    def generic(st):  # one multiply-add per stencil tap, one add per window element, point ops 1 (clamp 2)
        if st[0] == "point":
            return 2 if st[1] == "clamp" else 1
        return (2 * st[1] + 1) * (2 * st[2] + 1)
    return sum(generic(o) if isinstance(o, tuple) else table[o] for o in ops)


def time_plan(plan, x, bufs, steps, warmup, stream):
    """ms per run: `steps` runs back to back after `warmup`, bracketed by
    synchronisations and one pair of HIP events on `stream` (total / steps);
    then the same runs again with an event pair around each, whose median is
    reported beside it."""
    import torch
    out, pts, cnt, ws = bufs
    for _ in range(warmup):
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    mean = ev0.elapsed_time(ev1) / steps
    per = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
        b.record(stream)
        per.append((a, b))
    torch.cuda.synchronize()
    times = [a.elapsed_time(b) for a, b in per]
    return float(mean), float(np.median(times)), times


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


def cpu_baseline(wl, ops, budget_s=15.0):
    """The oracle (FP64, unfused) on a bounded sample of the same workload."""
    import oracle
    from paper_1509_04394_amd import synth
    oracle.build(force=False)
    cores = os.cpu_count() or 1
    W, H = wl["W"], wl["H"]
    n = 8
    generic = any(isinstance(o, tuple) for o in ops)
    run = (lambda v, k: oracle.gchain(ops, v, nthreads=k)) if generic else (lambda v, k: oracle.chain(ops, v, nthreads=k))
    vol = synth.video(W, H, n, seed=wl["seed"], rgb=wl["rgb"])
    t = time.perf_counter()
    run(vol, cores)
    dt = time.perf_counter() - t
    # grow the sample to about budget_s of work
    frames = int(min(wl["T"], max(n, n * budget_s / max(dt, 1e-3))))
    frames = max(cores, frames - frames % cores) if frames >= cores else frames
    vol = synth.video(W, H, frames, seed=wl["seed"], rgb=wl["rgb"])
    t = time.perf_counter()
    run(vol, min(cores, frames))
    dt = time.perf_counter() - t
    px = W * H * frames
    return {"value": px / dt / 1e6, "unit": "Mpixel/s", "cores": min(cores, frames), "kind": "oracle",
            "sample": f"frames 0-{frames - 1} of the {W}x{H}x{wl['T']} workload ({px / 1e6:.1f} Mpx), "
                      f"whole chain unfused in FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed runs first (the GPU clock rises over the first ~10 ms of load)")
    ap.add_argument("--workload", default="rgb800", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--engine", default="auto", choices=["auto", "tile", "row"],
                    help="kernel family for the fused plan's groups (auto: the planner's choice)")
    ap.add_argument("--autotune", action="store_true",
                    help="measure every band / tile configuration of each fused group first (untimed) and "
                         "keep the fastest")
    ap.add_argument("--no-unfused", action="store_true", help="skip timing the unfused sequence")
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
    tuned = None
    if args.autotune:
        from paper_1509_04394_amd import autotune
        tuned = autotune.autotune(fused, x, reps=3)
        log("autotuned", tuned)
    info = fused.segment_info()
    fb = fused.alloc(dev)
    log("fused plan groups", fused.segments, "tiles", [(s.tile_w, s.tile_h, s.frames_per_block) for s in info])
    f_mean, f_med, _ = time_plan(fused, x, fb, args.steps, args.warmup, stream)
    nfused = int(fb[2].item()) if fb[2] is not None else 0
    log(f"fused: {f_mean:.4f} ms/step back to back, {f_med:.4f} median with events around each run, "
        f"{nfused} points")
    pcie = None
    if not args.fused_only:
        e2e, h2d = pcie_inclusive(fused, x, fb, stream)
        pcie = {"ms_per_step": round(e2e, 4), "mpx_s": round(npx / (e2e * 1e-3) / 1e6, 1),
                "h2d_ms": round(h2d, 4), "h2d_GBs": round(x.numel() * x.element_size() / (h2d * 1e-3) / 1e9, 1),
                "note": "input copied from pinned host memory inside the timed pass; not the headline value"}
        log(f"with the host-to-device copy: {e2e:.3f} ms/step ({h2d:.3f} ms copy)")
    copy_gbs = None if args.fused_only else copy_ceiling_gbs(dev)

    unf = None
    if not (args.no_unfused or args.fused_only):
        del fb
        torch.cuda.empty_cache()
        uplan = fz.Plan(ops, W, H, T, partition="unfused", engine=args.engine)
        ub = uplan.alloc(dev)
        u_mean, u_med, _ = time_plan(uplan, x, ub, max(3, args.steps // 2), 1, stream)
        log(f"unfused: {u_mean:.3f} ms/step mean, {u_med:.3f} median")
        unf = {"mpx_s": npx / (u_mean * 1e-3) / 1e6, "ms_per_step": u_mean,
               "algorithmic_GBs": uplan.cost / (u_mean * 1e-3) / 1e9,
               "hbm_frac": uplan.cost / (u_mean * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "kernels": len(uplan.segments)}
        del ub
        torch.cuda.empty_cache()

    value = npx / (f_mean * 1e-3) / 1e6
    alg_bytes = fused.cost  # compulsory bytes of the planned groups
    dominant = info[0] if len(info) == 1 else max(info, key=lambda s: s.cost)
    opx = ops_per_px(ops[dominant.first:dominant.last + 1])
    achieved_gops = npx * opx / (f_mean * 1e-3) / 1e9
    achieved_gbs = alg_bytes / (f_mean * 1e-3) / 1e9
    traffic = None
    ct = COUNTER_TRAFFIC.get((args.workload, kernel_source_hash(),
                              (dominant.tile_w, dominant.tile_h, dominant.frames_per_block)))
    if ct is not None and dominant.engine == fz.FZ_ENGINE_ROW:
        # measured HBM bytes per launch over this run's launch time, GB/s
        traffic = round((ct["fetch_bytes"] + ct["write_bytes"]) / (f_mean * 1e-3) / 1e9, 1)
    roof = {"bound": "alu", "achieved": round(achieved_gops, 1), "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
            "frac": round(achieved_gops / VALU_PEAK_GOPS, 4), "traffic": traffic,
            "traffic_unit": "GB/s (counter bytes per launch / launch time)",
            "ops_per_px": opx, "hbm_achieved_GBs": round(achieved_gbs, 1),
            "hbm_frac": round(achieved_gbs / HBM_PEAK_GBS, 4)}
    rec = {"metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(f_mean, 4), "ms_per_step_events_each": round(f_med, 4),
           "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["desc"], "partition": fused.segments,
                      "tile": [dominant.tile_w, dominant.tile_h, dominant.frames_per_block],
                      "engine": {fz.FZ_ENGINE_ROW: "row", fz.FZ_ENGINE_TILE: "tile",
                                 fz.FZ_ENGINE_STREAM: "stream"}[dominant.engine],
                      "sizing": "autotuned" if args.autotune else "planner",
                      "points_per_step": nfused},
           "roofline": roof}
    if copy_gbs is not None:
        # the same bytes against a plain device copy measured in this run
        rec["copy_ceiling_GBs"] = round(copy_gbs, 1)
        roof["hbm_frac_of_copy"] = round(achieved_gbs / copy_gbs, 4)
        if unf is not None:
            unf["hbm_frac_of_copy"] = unf["algorithmic_GBs"] / copy_gbs
    if pcie is not None:
        rec["pcie_inclusive"] = pcie
    if unf is not None:
        rec["unfused"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in unf.items()}
        rec["speedup_vs_unfused"] = round(u_mean / f_mean, 3)
        rec["paper_context"] = "2-3x fused over sequential kernels on Tesla C1060 / K20 / GTX 750 Ti (Abstract)"
    if not (args.no_cpu or args.fused_only):
        log("timing the CPU oracle on a sample")
        rec["cpu_baseline"] = cpu_baseline(wl, ops)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
