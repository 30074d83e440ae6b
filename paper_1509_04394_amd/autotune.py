"""Measured tile / band sizing of a plan's groups.

The paper sizes a fused kernel's box from the data-utilisation model (Eq. 3-6)
and benchmarks box sizes (Sec. VIII, Fig. 9).  Here each group of a plan is
timed in every configuration the library compiles -- the LDS tile engine with
each tile, the row-marching engine with a range of band heights and frames per
work item -- on the plan's real intermediate inputs, and the fastest is set on
the plan (fz_plan_set_segment_config).  All device work runs through the C ABI.
"""
from __future__ import annotations

import numpy as np

from . import fz

TILES = [(64, 16), (32, 32), (64, 32)]
BANDS = [32, 44, 55, 67, 86, 100, 150]
FRAME_RUNS = [8, 12, 16, 24]


def candidates(info):
    """Configurations to try for a group described by fz_segment_info."""
    if info.engine == fz.FZ_ENGINE_STREAM:
        return []
    c = [dict(engine="tile", tile_w=w, tile_h=h) for (w, h) in TILES]
    if info.engine == fz.FZ_ENGINE_ROW:
        runs = FRAME_RUNS if info.halo_t > 0 else [0]
        c += [dict(engine="row", tile_h=b, frames_per_block=t) for b in BANDS for t in runs]
    return c


def _time(plan, x, reps):
    import torch
    out, pts, cnt, ws = plan.alloc(x.device, point_capacity=1 << 20)
    s = torch.cuda.current_stream(x.device)
    plan.run(x, out, pts, cnt, ws, stream=s.cuda_stream)
    ev = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        plan.run(x, out, pts, cnt, ws, stream=s.cuda_stream)
        b.record(s)
        ev.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def autotune(plan: "fz.Plan", x, reps=5, log=None):
    """Tune every group of `plan` (a fz.Plan) on input tensor x in place; returns
    [(group, best config, best ms, default ms)]."""
    import torch
    ops, W, H, T = plan.ops, plan.W, plan.H, plan.T
    # inputs of each group: run the plan's own prefix
    ins = {}
    cur = x
    infos = plan.segment_info()
    for i, s in enumerate(infos):
        ins[i] = cur
        if i + 1 < len(infos):
            sub = fz.Plan(ops[:s.last + 1], W, H, T, partition=plan.segments[:i])
            cur, _, _ = sub.run(x)
    torch.cuda.synchronize()
    report = []
    for i, s in enumerate(infos):
        sub_ops = ops[s.first:s.last + 1]
        base = fz.Plan(sub_ops, W, H, T, partition=[])
        default_ms = _time(base, ins[i], reps)
        best = (None, default_ms)
        for cfg in candidates(s):
            try:
                trial = fz.Plan(sub_ops, W, H, T, partition=[])
                fz.fz_plan_set_segment_config(trial.handle, 0, **cfg)
            except fz.FzError:
                continue
            ms = _time(trial, ins[i], reps)
            if log:
                log(f"[autotune] group {s.first}..{s.last} {cfg}: {ms:.3f} ms")
            if ms < best[1]:
                best = (cfg, ms)
        if best[0] is not None:
            fz.fz_plan_set_segment_config(plan.handle, i, **best[0])
        report.append(((s.first, s.last), best[0], best[1], default_ms))
    return report
