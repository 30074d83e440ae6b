"""Measured tile / band sizing of a plan's groups.

The paper sizes a fused kernel's box from the data-utilisation model (Eq. 3-6)
and benchmarks box sizes (Sec. VIII, Fig. 9).  Here each group of a plan is
timed in the configurations the library compiles -- the LDS tile engine with
each tile, the row-marching engine with a range of band heights and frames
per work item around the Eq. 6 seed -- on the plan's real intermediate
inputs, and the fastest is set on the plan (fz_plan_set_segment_config).
All device work runs through the C ABI.
"""
from __future__ import annotations

import math

import numpy as np

from . import fz

TILES = [(64, 16), (32, 32), (64, 32)]
BANDS = [32, 44, 55, 67, 86, 100, 150]
FRAME_RUNS = [1, 2, 4, 8, 16]
ROW_SLOTS = 256 * 4 * 5  # wavefronts the device holds at once (5 per SIMD, the RGB row kernel)
ROW_HALO, ROW_SPAN = 6, 128  # rows of halo per band side; columns per strip (64 lanes x 2)


def eq6_row(beta, dy, dt):
    """Eq. 6 for the row kernel's box: its strips have a fixed width, so only
    the band height y and the frame run t are free.  Of the boxes with
    y * t = beta output rows x frames, the one whose input box
    (y + 2 dy)(t + dt) is least: y = sqrt(2 dy beta / dt), t = sqrt(dt beta / (2 dy))
    (the same derivation as Eq. 6, with one spatial axis instead of two)."""
    if dt <= 0:
        return beta, 1.0
    if dy <= 0:
        return 1.0, beta
    return math.sqrt(2.0 * dy * beta / dt), math.sqrt(dt * beta / (2.0 * dy))


def row_seed(W, H, T, halo_t):
    """(band rows, frames) seed for a row-engine group of a W x H x T video: the
    work of one full round of wavefronts per work item, beta = H T nstrips /
    ROW_SLOTS rows x frames, through eq6_row with the row kernel's halos."""
    S = ROW_SPAN - 2 * ROW_HALO
    nstrips = 1 + max(0, -(-(W - ROW_SPAN) // S))
    beta = max(1.0, H * T * nstrips / ROW_SLOTS)
    y, t = eq6_row(beta, ROW_HALO, max(halo_t, 0))
    return int(min(max(round(y), 8), H)), int(min(max(round(t), 1), T))


def candidates(info, W=None, H=None, T=None):
    """Configurations to try for a group described by fz_segment_info: every
    compiled tile; for a row-engine group, band heights x frame runs from the
    fixed lists and around the Eq. 6 seed (when the video size is given)."""
    if info.engine == fz.FZ_ENGINE_STREAM:
        return []
    c = [dict(engine="tile", tile_w=w, tile_h=h) for (w, h) in TILES]
    if info.engine == fz.FZ_ENGINE_ROW:
        bands, runs = list(BANDS), list(FRAME_RUNS) if info.halo_t > 0 else [0]
        if W is not None:
            y, t = row_seed(W, H, T, info.halo_t)
            bands += [max(8, int(y * f)) for f in (0.5, 0.75, 1.0, 1.5)]
            if info.halo_t > 0:
                runs += [max(1, int(round(t * f))) for f in (0.5, 1.0, 2.0)]
        bands = sorted(set(b for b in bands if b <= max(H or 10 ** 9, 8)))
        runs = sorted(set(runs))
        c += [dict(engine="row", tile_h=b, frames_per_block=t) for b in bands for t in runs]
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


def autotune(plan: "fz.Plan", x, reps=5, log=None, stats=None):
    """Tune every group of `plan` (a fz.Plan) on input tensor x in place; returns
    [(group, best config, best ms, default ms)].  A configuration is kept only
    when it beats the planner's by more than 1% (timing noise).  stats (a
    dict), if given, receives the number of configurations timed ("tried")."""
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
        for cfg in candidates(s, W, H, T):
            try:
                trial = fz.Plan(sub_ops, W, H, T, partition=[])
                fz.fz_plan_set_segment_config(trial.handle, 0, **cfg)
            except fz.FzError:
                continue
            ms = _time(trial, ins[i], reps)
            if stats is not None:
                stats["tried"] = stats.get("tried", 0) + 1
            if log:
                log(f"[autotune] group {s.first}..{s.last} {cfg}: {ms:.3f} ms")
            if ms < best[1] * (0.99 if best[0] is None else 1.0):
                best = (cfg, ms)
        if best[0] is not None:
            fz.fz_plan_set_segment_config(plan.handle, i, **best[0])
        report.append(((s.first, s.last), best[0], best[1], default_ms))
    return report
