"""Learned group prices.

The paper prices each candidate fused kernel by its predicted execution time
C_i and picks the partition of least total (Sec. VI, Fig. 5).  Here the
prediction is learned from the planner's own kernels:

* ``measure_table``: every contiguous group of a chain, in every kernel
  configuration the planner may choose (row-marching, LDS tile with each
  compiled tile, streaming), is timed on the GPU with HIP events on real
  intermediate inputs; each sample is (group features, microseconds);
* ``train``: the library's HIP kernels (``fz_mlp_loss_grad``, ``fz_mlp_adam_step``)
  fit the cost network to log(microseconds), full batch, Adam;
* ``evaluate_case``: the partitions chosen with learned prices and with the
  analytic (bytes) prices, timed from the measured table, against the best
  partition under measured prices (exact DP over the table).

All device work goes through the C ABI; torch only provides memory and streams.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import fz, synth

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "cost_weights.json")
FRAME_SIZES = [(192, 432), (320, 240), (640, 480), (800, 600)]
CHAINS = {"rgb_harris": fz.RGB_HARRIS_CHAIN, "harris": fz.HARRIS_CHAIN, "grad": fz.GRAD_CHAIN}
TILES = [(64, 16), (32, 32), (64, 32)]


def _is_window(op):
    if isinstance(op, tuple):
        return op[0] != "point"
    return op in ("gauss5", "sobel3", "boxsum5", "nms3")


def _in_dtype(ops, a):
    """Input type of a generic group starting at stage a (u8 video or f32 intermediate)."""
    return "u8" if a == 0 else "f32"


def group_configs(ops, a, b):
    """Kernel configurations of group a..b: the planner's automatic choice and
    every compiled LDS tile (groups with a window stage)."""
    window = any(_is_window(op) for op in ops[a:b + 1])
    cfgs = [dict(engine="auto")]
    if window:
        cfgs += [dict(engine="tile", tile=t) for t in TILES]
    return cfgs


def _inputs(ops, W, H, T, seed, dev):
    """Real inputs of every stage: the video, then each prefix's output."""
    import torch
    rgb = ops[0] == "rgb2gray"
    vid = torch.from_numpy(synth.video(W, H, T, seed=seed, rgb=rgb)).to(dev)
    ins = [vid]
    for a in range(1, len(ops)):
        plan = fz.Plan(ops[:a], W, H, T)  # generic chains: u8 video in, f32 out
        out, pts, cnt = plan.run(vid)
        ins.append(out)
    torch.cuda.synchronize()
    return ins


def _time_plan(plan, x, reps):
    import torch
    out, pts, cnt, ws = plan.alloc(x.device, point_capacity=1 << 20)
    stream = torch.cuda.current_stream(x.device)
    plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.run(x, out, pts, cnt, ws, stream=stream.cuda_stream)
        e1.record(stream)
        times.append((e0, e1))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in times])) * 1e3  # microseconds


def measure_table(ops, W, H, T, seed=0, reps=5, dev=None):
    """{(a, b, engine, tile_w, tile_h): (features, microseconds)} for every group
    and configuration (keys use the configuration the plan actually got)."""
    import torch
    dev = dev or torch.device("cuda:0")
    ins = _inputs(ops, W, H, T, seed, dev)
    table = {}
    n = len(ops)
    for a in range(n):
        for b in range(a, n):
            for cfg in group_configs(ops, a, b):
                extra = {"in_dtype": _in_dtype(ops, a)} if isinstance(ops[0], tuple) else {}
                try:
                    plan = fz.Plan(ops[a:b + 1], W, H, T, partition=[], **cfg, **extra)
                except fz.FzError:
                    continue
                s = plan.segment_info()[0]
                key = (a, b, int(s.engine), int(s.tile_w), int(s.tile_h))
                if key in table:
                    continue
                us = _time_plan(plan, ins[a], reps)
                feats = fz.fz_plan_segment_features(plan.handle, 0)
                table[key] = (feats, us)
    del ins
    torch.cuda.empty_cache()
    return table


def table_rows(table):
    X = np.array([f for f, _ in table.values()], np.float32)
    y = np.array([math.log(us) for _, us in table.values()], np.float32)
    return X, y


# ---------------------------------------------------------------- training
def init_params(F, seed):
    rng = np.random.default_rng(seed)
    H = 64
    W1 = rng.normal(0, math.sqrt(2.0 / F), (H, F))
    W2 = rng.normal(0, math.sqrt(2.0 / H), (H, H))
    W3 = rng.normal(0, math.sqrt(1.0 / H), H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.full(H, 0.01), W3, [0.0]]).astype(np.float32)


def train(X, y, steps=4000, lr=3e-3, seed=0, log_every=0):
    """Full-batch Adam with the library's GPU kernels; returns (params, losses)."""
    import torch
    dev = torch.device("cuda:0")
    F = X.shape[1]
    n = X.shape[0]
    P = fz.fz_mlp_param_count(F)
    p0 = init_params(F, seed)
    p0[-1] = float(np.mean(y))  # start the output bias at the mean target
    dp = torch.tensor(p0, device=dev)
    dx = torch.tensor(X, device=dev)
    dt = torch.tensor(y, device=dev)
    g = torch.empty(P, device=dev)
    L = torch.empty(1, device=dev)
    m = torch.zeros(P, device=dev)
    v = torch.zeros(P, device=dev)
    ws = torch.empty(fz.fz_mlp_workspace_bytes(F, n), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    losses = []
    for step in range(1, steps + 1):
        fz.fz_mlp_loss_grad(dp.data_ptr(), F, dx.data_ptr(), dt.data_ptr(), n, g.data_ptr(), L.data_ptr(),
                            ws.data_ptr(), ws.numel(), s)
        fz.fz_mlp_adam_step(dp.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), P, step, lr, 0.9, 0.999, 1e-8,
                            s)
        if step % 50 == 0 or step == 1:
            losses.append((step, L.item()))
            if log_every and step % log_every == 0:
                print(f"[costmodel] step {step} loss {losses[-1][1]:.5f}", flush=True)
    return dp.cpu().numpy(), losses


def predict(params, X):
    import torch
    dev = torch.device("cuda:0")
    X = np.asarray(X, np.float32)
    y = torch.empty(X.shape[0], device=dev)
    dp = torch.tensor(np.asarray(params, np.float32), device=dev)  # alive until the kernel has run
    dx = torch.tensor(X, device=dev)
    fz.fz_mlp_forward(dp.data_ptr(), X.shape[1], dx.data_ptr(), X.shape[0], y.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
    return y.cpu().numpy()


def save_weights(params, meta, path=WEIGHTS_PATH):
    with open(path, "w") as f:
        json.dump({"n_features": fz.fz_cost_n_features(), "params": [float(v) for v in params], "meta": meta}, f)


def load_weights(path=WEIGHTS_PATH):
    with open(path) as f:
        d = json.load(f)
    if d["n_features"] != fz.fz_cost_n_features():
        raise ValueError("cost weights were trained for another feature set")
    return np.array(d["params"], np.float32), d.get("meta", {})


# ---------------------------------------------------------------- evaluation
def plan_time(plan, table):
    """Measured time of a plan's groups in the configurations it chose."""
    total = 0.0
    for s in plan.segment_info():
        key = (s.first, s.last, int(s.engine), int(s.tile_w), int(s.tile_h))
        if key not in table:
            raise KeyError(f"configuration {key} was not measured")
        total += table[key][1]
    return total


def best_measured(ops, table):
    """Least total measured time over every partition and configuration (exact DP)."""
    n = len(ops)
    c = [[math.inf] * n for _ in range(n)]
    for (a, b, *_), (_, us) in table.items():
        c[a][b] = min(c[a][b], us)
    total, seg_last = fz.fz_partition_min(c)
    return total, seg_last


def evaluate_case(ops, W, H, T, params, table):
    best, best_part = best_measured(ops, table)
    learned = fz.Plan(ops, W, H, T, cost_weights=params)
    analytic = fz.Plan(ops, W, H, T)
    tl, ta = plan_time(learned, table), plan_time(analytic, table)
    return {"W": W, "H": H, "T": T, "n": len(ops), "best_us": best, "best_partition": best_part,
            "learned_us": tl, "learned_partition": learned.segments,
            "analytic_us": ta, "analytic_partition": analytic.segments,
            "learned_ratio": tl / best, "analytic_ratio": ta / best}


def cases(seed, n_cases):
    """Seeded (chain name, W, H, T) workloads of the fixed chains."""
    rng = np.random.default_rng(seed)
    out = []
    names = sorted(CHAINS)
    for _ in range(n_cases):
        name = names[int(rng.integers(0, len(names)))]
        W, H = FRAME_SIZES[int(rng.integers(0, len(FRAME_SIZES)))]
        T = int(rng.choice([8, 24, 64, 160]))
        out.append((name, W, H, T))
    return out


RANDOM_T = 64


def random_cases(first_seed, n_cases):
    """Random generic chains: chain k drawn by synth.random_chain(first_seed + k),
    frame size uniform over FRAME_SIZES (from the same seed), 64 frames.  Each
    case is ("random:<seed>", W, H, T)."""
    out = []
    for k in range(n_cases):
        sd = first_seed + k
        W, H = FRAME_SIZES[int(np.random.default_rng([sd, 1]).integers(0, len(FRAME_SIZES)))]
        out.append((f"random:{sd}", W, H, RANDOM_T))
    return out


def case_ops(name):
    """Stage list of a case name: a fixed chain or a random generic chain."""
    if name.startswith("random:"):
        return synth.random_chain(int(name.split(":")[1]))
    return CHAINS[name]


def build(n_train=24, n_test=8, seed=5, steps=4000, out=WEIGHTS_PATH, log=print, n_random_train=0,
          n_random_test=0, reps=5):
    """Measure, train and evaluate; write the weights (with the evaluation) to `out`.
    Random generic chains are seeded from 5000 (training) and 9000 (test)."""
    t0 = time.time()
    train_cases = cases(seed, n_train) + random_cases(5000, n_random_train)
    test_cases = cases(seed + 1000, n_test) + random_cases(9000, n_random_test)
    X, y = [], []
    for i, (name, W, H, T) in enumerate(train_cases):
        tab = measure_table(case_ops(name), W, H, T, seed=seed + i, reps=reps)
        Xi, yi = table_rows(tab)
        X.append(Xi)
        y.append(yi)
        log(f"[costmodel] train case {i} {name} {W}x{H}x{T}: {len(yi)} samples ({time.time() - t0:.0f} s)")
    X = np.concatenate(X)
    y = np.concatenate(y)
    params, losses = train(X, y, steps=steps, seed=seed)
    train_rmse = float(np.sqrt(np.mean((predict(params, X) - y) ** 2)))
    log(f"[costmodel] trained on {len(y)} samples, rmse(log us) {train_rmse:.4f}")
    evals = []
    Xt, yt = [], []
    for j, (name, W, H, T) in enumerate(test_cases):
        ops = case_ops(name)
        tab = measure_table(ops, W, H, T, seed=seed + 5000 + j, reps=reps)
        Xi, yi = table_rows(tab)
        Xt.append(Xi)
        yt.append(yi)
        r = evaluate_case(ops, W, H, T, params, tab)
        r["chain"] = name
        evals.append(r)
        log(f"[costmodel] test {name} {W}x{H}x{T}: learned {r['learned_ratio']:.3f} analytic "
            f"{r['analytic_ratio']:.3f} of best")
    Xt = np.concatenate(Xt)
    yt = np.concatenate(yt)
    test_rmse = float(np.sqrt(np.mean((predict(params, Xt) - yt) ** 2)))
    geo = lambda k, rs=None: float(np.exp(np.mean([math.log(r[k]) for r in (evals if rs is None else rs)])))
    rnd = [r for r in evals if r["chain"].startswith("random:")]
    fixed = [r for r in evals if not r["chain"].startswith("random:")]
    meta = {"train_samples": int(len(y)), "test_samples": int(len(yt)), "train_rmse_log_us": train_rmse,
            "test_rmse_log_us": test_rmse, "steps": steps, "final_loss": losses[-1][1],
            "train_cases": train_cases, "test_cases": test_cases, "evaluation": evals,
            "geomean_learned_over_best": geo("learned_ratio"), "geomean_analytic_over_best": geo("analytic_ratio"),
            "seconds": time.time() - t0}
    for tag, rs in (("random", rnd), ("fixed", fixed)):
        if rs:
            meta[f"geomean_learned_over_best_{tag}"] = geo("learned_ratio", rs)
            meta[f"geomean_analytic_over_best_{tag}"] = geo("analytic_ratio", rs)
    save_weights(params, meta, out)
    log(f"[costmodel] geomean learned/best {meta['geomean_learned_over_best']:.4f}, "
        f"analytic/best {meta['geomean_analytic_over_best']:.4f}; test rmse {test_rmse:.4f}")
    return params, meta


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="measure group times, train the cost network, evaluate")
    ap.add_argument("out", nargs="?", default=WEIGHTS_PATH)
    ap.add_argument("--fixed-train", type=int, default=24)
    ap.add_argument("--fixed-test", type=int, default=8)
    ap.add_argument("--random-train", type=int, default=0)
    ap.add_argument("--random-test", type=int, default=0)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    build(n_train=a.fixed_train, n_test=a.fixed_test, n_random_train=a.random_train, n_random_test=a.random_test,
          steps=a.steps, reps=a.reps, out=a.out, log=lambda m: print(m, flush=True))
