"""Learned group prices.

The paper prices each candidate fused kernel by its predicted execution time
C_i and picks the partition of least total (Sec. VI, Fig. 5).  Here the
prediction is learned from the planner's own kernels:

* ``measure_table``: every contiguous group of a chain, in every kernel
  configuration the planner may choose (row-marching, LDS tile with each
  compiled tile, streaming), is timed on the GPU with HIP events on real
  intermediate inputs; each sample is (group features, microseconds);
* ``train_mlp``: the library's HIP kernels (``fz_mlp_loss_grad``, ``fz_mlp_adam_step``)
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


def train_mlp(X, y, steps=4000, lr=3e-3, seed=0, log_every=0, batch=0, X_val=None, y_val=None, eval_every=250,
              p_init=None):
    """Adam with the library's GPU kernels: full batch (batch = 0) or mini-batches
    of `batch` rows drawn from a seeded shuffle, from a seeded initialisation or
    from `p_init`.  With a validation set, the parameters of least validation
    loss (checked every `eval_every` steps) are returned.  Returns (params,
    {"best_step", "val": [(step, loss)]})."""
    import torch
    dev = torch.device("cuda:0")
    F = X.shape[1]
    n = X.shape[0]
    P = fz.fz_mlp_param_count(F)
    if p_init is not None:
        p0 = np.array(p_init, np.float32)
    else:
        p0 = init_params(F, seed)
        p0[-1] = float(np.mean(y))  # start the output bias at the mean target
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n) if batch else np.arange(n)
    dp = torch.tensor(p0, device=dev)
    dx = torch.tensor(np.ascontiguousarray(X[perm]), device=dev)
    dt = torch.tensor(np.ascontiguousarray(y[perm]), device=dev)
    B = min(batch, n) if batch else n
    g = torch.empty(P, device=dev)
    L = torch.empty(1, device=dev)
    m = torch.zeros(P, device=dev)
    v = torch.zeros(P, device=dev)
    ws = torch.empty(fz.fz_mlp_workspace_bytes(F, B), dtype=torch.uint8, device=dev)
    if X_val is not None:
        dxv = torch.tensor(np.asarray(X_val, np.float32), device=dev)
        dyv = torch.tensor(np.asarray(y_val, np.float32), device=dev)
        gv = torch.empty(P, device=dev)
        Lv = torch.empty(1, device=dev)
        wsv = torch.empty(fz.fz_mlp_workspace_bytes(F, dxv.shape[0]), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    nb = max(1, n // B)
    best, best_step, curve = None, 0, []
    for step in range(1, steps + 1):
        off = ((step - 1) % nb) * B
        fz.fz_mlp_loss_grad(dp.data_ptr(), F, dx[off:off + B].data_ptr(), dt[off:off + B].data_ptr(), B,
                            g.data_ptr(), L.data_ptr(), ws.data_ptr(), ws.numel(), s)
        fz.fz_mlp_adam_step(dp.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), P, step, lr, 0.9, 0.999, 1e-8,
                            s)
        if X_val is not None and (step % eval_every == 0 or step == steps):
            fz.fz_mlp_loss_grad(dp.data_ptr(), F, dxv.data_ptr(), dyv.data_ptr(), dxv.shape[0], gv.data_ptr(),
                                Lv.data_ptr(), wsv.data_ptr(), wsv.numel(), s)
            lv = Lv.item()
            curve.append((step, lv))
            if best is None or lv < best[0]:
                best = (lv, dp.clone())
                best_step = step
            if log_every:
                print(f"[costmodel] step {step} val loss {lv:.5f}", flush=True)
        elif log_every and step % log_every == 0:
            print(f"[costmodel] step {step} loss {L.item():.5f}", flush=True)
    params = (best[1] if best is not None else dp).cpu().numpy()
    return params, {"best_step": best_step if best is not None else steps, "val": curve}


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


def save_table(path, case, table):
    """Write one case's measured table (.npz: configuration keys, features, microseconds)."""
    keys = np.array([list(k) for k in table], np.int32).reshape(-1, 5)
    feats = np.array([f for f, _ in table.values()], np.float32).reshape(len(table), -1)
    us = np.array([u for _, u in table.values()], np.float64)
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, case=np.array([str(c) for c in case]), keys=keys, feats=feats, us=us,
                        n_features=np.int32(fz.fz_cost_n_features()))
    os.replace(tmp, path)


def load_table(path):
    d = np.load(path, allow_pickle=False)
    if int(d["n_features"]) != fz.fz_cost_n_features():
        raise ValueError(f"{path}: measured for another feature set")
    c = [str(v) for v in d["case"]]
    case = (c[0], int(c[1]), int(c[2]), int(c[3]))
    table = {tuple(int(v) for v in k): (list(map(float, f)), float(u))
             for k, f, u in zip(d["keys"], d["feats"], d["us"])}
    return case, table


def campaign():
    """The measured workloads, split by chain: training = the fixed chains at 24
    seeded sizes and 4000 random generic chains (seeds 5000..8999); validation =
    500 random chains (9000..9499), used to pick the number of training steps;
    test = the fixed chains at 8 other sizes and 500 random chains (9500..9999)."""
    return {"train": cases(5, 24) + random_cases(5000, 4000),
            "val": random_cases(9000, 500),
            "test": cases(1005, 8) + random_cases(9500, 500)}


# Fixed-chain sizes: a grid for training, and held-out (chain, W, H, T) tuples
# that the grid never contains (frame counts off the grid), for the tests.
FIXED_T_GRID = [8, 16, 32, 64, 128, 256, 512, 1000]
FIXED_HELD_OUT = [("rgb_harris", 640, 480, 40), ("harris", 320, 240, 100), ("grad", 800, 600, 48),
                  ("rgb_harris", 192, 432, 90), ("harris", 800, 600, 20), ("grad", 640, 480, 150),
                  ("harris", 192, 432, 300), ("rgb_harris", 320, 240, 200), ("rgb_harris", 800, 600, 700),
                  ("harris", 640, 480, 600)]


def fixed_campaign():
    """Fixed chains: training = every chain at the four frame sizes and the
    frame counts of FIXED_T_GRID; test = FIXED_HELD_OUT (sizes off the grid)."""
    train = [(c, W, H, T) for c in sorted(CHAINS) for (W, H) in FRAME_SIZES for T in FIXED_T_GRID]
    held = set(FIXED_HELD_OUT)
    assert not held & set(train)
    return {"train": train, "test": list(FIXED_HELD_OUT)}


def forward_np(params, X):
    """The cost network on the host in FP64 (numpy), parameter layout of fz_mlp_forward."""
    X = np.asarray(X, np.float64)
    F, Hd = X.shape[1], 64
    p = np.asarray(params, np.float64)
    o = 0
    W1 = p[o:o + Hd * F].reshape(Hd, F); o += Hd * F
    b1 = p[o:o + Hd]; o += Hd
    W2 = p[o:o + Hd * Hd].reshape(Hd, Hd); o += Hd * Hd
    b2 = p[o:o + Hd]; o += Hd
    W3 = p[o:o + Hd]; o += Hd
    b3 = p[o]
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3 + b3


def group_feature_rows(ops, W, H, T):
    """Features of every contiguous group of a chain in every configuration
    (host only: planning needs no device)."""
    rows = []
    n = len(ops)
    for a in range(n):
        for b in range(a, n):
            for cfg in group_configs(ops, a, b):
                extra = {"in_dtype": _in_dtype(ops, a)} if isinstance(ops[0], tuple) else {}
                try:
                    plan = fz.Plan(ops[a:b + 1], W, H, T, partition=[], **cfg, **extra)
                except fz.FzError:
                    continue
                rows.append(fz.fz_plan_segment_features(plan.handle, 0))
    return np.array(rows, np.float32).reshape(-1, fz.fz_cost_n_features())


def distill_rows(params, first_seed, n_chains):
    """Features of the random generic chains' groups (the random workload of the
    original training, seeds first_seed..), labelled by the current network:
    fine-tuning on measured fixed-chain times keeps what the network learned
    of random chains by fitting its own predictions there."""
    X = np.concatenate([group_feature_rows(case_ops(name), W, H, T)
                        for name, W, H, T in random_cases(first_seed, n_chains)])
    return X, forward_np(params, X).astype(np.float32)


def measure_fixed(directory, split, reps=5, log=print):
    """Measure the fixed-chain campaign split into directory/fixed_<split>_NNNN.npz."""
    os.makedirs(directory, exist_ok=True)
    todo = fixed_campaign()[split]
    t0 = time.time()
    for i, (name, W, H, T) in enumerate(todo):
        path = os.path.join(directory, f"fixed_{split}_{i:04d}.npz")
        if os.path.exists(path):
            continue
        tab = measure_table(case_ops(name), W, H, T, seed=60000 + 1000 * (split == "test") + i, reps=reps)
        save_table(path, todo[i], tab)
        log(f"[costmodel] fixed {split} {i} {name} {W}x{H}x{T}: {len(tab)} samples ({time.time() - t0:.0f} s)")


def finetune_fixed(directory, params0, meta0, steps=3000, batch=4096, distill_chains=400, fixed_weight=4,
                   out=WEIGHTS_PATH, log=print):
    """Fine-tune the network on measured fixed-chain times (training grid),
    replicated `fixed_weight` times, together with distillation rows that hold
    its random-chain predictions; keep the step of least loss on the held-out
    fixed cases' measured rows; evaluate plan quality on the held-out fixed
    cases and on any measured random test tables in the directory."""
    t0 = time.time()
    train = [load_table(os.path.join(directory, f)) for f in sorted(os.listdir(directory))
             if f.startswith("fixed_train_")]
    test = [load_table(os.path.join(directory, f)) for f in sorted(os.listdir(directory))
            if f.startswith("fixed_test_")]
    rtest = [load_table(os.path.join(directory, f)) for f in sorted(os.listdir(directory))
             if f.startswith("test_")]
    Xf, yf = _rows(train)
    Xd, yd = distill_rows(params0, 5000, distill_chains)
    X = np.concatenate([np.repeat(Xf, fixed_weight, axis=0), Xd])
    y = np.concatenate([np.repeat(yf, fixed_weight), yd])
    Xv, yv = _rows(test)
    params, curve = train_mlp(X, y, steps=steps, lr=1e-3, seed=11, batch=batch, X_val=Xv, y_val=yv,
                              eval_every=100, p_init=params0)
    rmse = lambda A, b: float(np.sqrt(np.mean((forward_np(params, A) - b) ** 2)))
    evals = []
    for (name, W, H, T), tab in test + rtest:
        r = evaluate_case(case_ops(name), W, H, T, params, tab)
        r["chain"] = name
        evals.append(r)
    geo = lambda rs: float(np.exp(np.mean([math.log(r["learned_ratio"]) for r in rs]))) if rs else None
    geo_a = lambda rs: float(np.exp(np.mean([math.log(r["analytic_ratio"]) for r in rs]))) if rs else None
    fixed = [r for r in evals if not r["chain"].startswith("random:")]
    rnd = [r for r in evals if r["chain"].startswith("random:")]
    meta = dict(meta0)
    meta["finetune"] = {
        "fixed_train_cases": len(train), "fixed_train_rows": int(len(yf)), "fixed_weight": fixed_weight,
        "distill_chains": distill_chains, "distill_rows": int(len(yd)), "steps": steps, "best_step": curve["best_step"],
        "rmse_log_us": {"fixed_train": rmse(Xf, yf), "fixed_test": rmse(Xv, yv), "distill": rmse(Xd, yd)},
        "held_out_fixed_cases": [list(c) for c, _ in test],
        "geomean_learned_over_best_fixed": geo(fixed), "geomean_analytic_over_best_fixed": geo_a(fixed),
        "worst_learned_over_best_fixed": max((r["learned_ratio"] for r in fixed), default=None),
        "geomean_learned_over_best_random": geo(rnd), "geomean_analytic_over_best_random": geo_a(rnd),
        "random_test_cases": len(rnd), "evaluation": evals, "seconds": time.time() - t0}
    save_weights(params, meta, out)
    log(f"[costmodel] fine-tuned: fixed held-out geomean learned {geo(fixed):.4f} (analytic {geo_a(fixed):.4f}), "
        f"random {geo(rnd) if rnd else float('nan'):.4f} over {len(rnd)} cases")
    return params, meta


def measure_cases(directory, split, first=0, count=None, reps=3, max_seconds=None, log=print):
    """Measure cases [first, first+count) of a campaign split into
    directory/<split>_NNNN.npz, skipping files that exist; stops starting new
    cases after max_seconds.  Returns True when the range is complete."""
    os.makedirs(directory, exist_ok=True)
    t0 = time.time()
    todo = campaign()[split]
    last = len(todo) if count is None else min(len(todo), first + count)
    base = {"train": 0, "val": 20000, "test": 40000}[split]
    done = 0
    for i in range(first, last):
        path = os.path.join(directory, f"{split}_{i:04d}.npz")
        if os.path.exists(path):
            continue
        if max_seconds is not None and time.time() - t0 > max_seconds:
            log(f"[costmodel] time budget reached at {split} {i}; {done} cases measured in this call")
            return False
        name, W, H, T = todo[i]
        tab = measure_table(case_ops(name), W, H, T, seed=5 + base + i, reps=reps)
        save_table(path, todo[i], tab)
        done += 1
        if done % 25 == 0 or i == last - 1:
            log(f"[costmodel] {split} {i} {name} {W}x{H}x{T}: {len(tab)} samples ({time.time() - t0:.0f} s)")
    return True


def _load_split(directory, split):
    files = sorted(f for f in os.listdir(directory) if f.startswith(split + "_") and f.endswith(".npz"))
    return [load_table(os.path.join(directory, f)) for f in files]


def _rows(tables):
    X = np.concatenate([table_rows(t)[0] for _, t in tables])
    y = np.concatenate([table_rows(t)[1] for _, t in tables])
    return X, y


def train_from_tables(directory, steps=6000, batch=8192, seed=5, out=WEIGHTS_PATH, log=print):
    """Train on the training split (mini-batch Adam on the GPU kernels), keep
    the parameters of least validation loss, evaluate plan quality on the test
    split, and write the weights with the evaluation to `out`."""
    t0 = time.time()
    train, val, test = (_load_split(directory, s) for s in ("train", "val", "test"))
    X, y = _rows(train)
    Xv, yv = _rows(val) if val else (X, y)
    params, curve = train_mlp(X, y, steps=steps, seed=seed, batch=batch, X_val=Xv, y_val=yv)
    rmse = lambda A, b: float(np.sqrt(np.mean((predict(params, A) - b) ** 2)))
    train_rmse, val_rmse = rmse(X, y), rmse(Xv, yv)
    log(f"[costmodel] {len(y)} training rows from {len(train)} chains; rmse(log us) train {train_rmse:.4f} "
        f"val {val_rmse:.4f} ({time.time() - t0:.0f} s)")
    evals = []
    for (name, W, H, T), tab in test:
        r = evaluate_case(case_ops(name), W, H, T, params, tab)
        r["chain"] = name
        evals.append(r)
    Xt, yt = _rows(test)
    test_rmse = rmse(Xt, yt)
    geo = lambda k, rs: float(np.exp(np.mean([math.log(r[k]) for r in rs])))
    worst = lambda k, rs: float(max(r[k] for r in rs))
    meta = {"train_chains": len(train), "val_chains": len(val), "test_chains": len(test),
            "train_rows": int(len(y)), "val_rows": int(len(yv)), "test_rows": int(len(yt)),
            "rmse_log_us": {"train": train_rmse, "val": val_rmse, "test": test_rmse},
            "steps": steps, "batch": batch, "best_step": curve["best_step"], "val_curve": curve["val"],
            "test_cases": [list(c) for c, _ in test], "evaluation": evals, "seconds": time.time() - t0}
    for tag, rs in (("all", evals), ("random", [r for r in evals if r["chain"].startswith("random:")]),
                    ("fixed", [r for r in evals if not r["chain"].startswith("random:")])):
        if rs:
            meta[f"geomean_learned_over_best_{tag}"] = geo("learned_ratio", rs)
            meta[f"geomean_analytic_over_best_{tag}"] = geo("analytic_ratio", rs)
            meta[f"worst_learned_over_best_{tag}"] = worst("learned_ratio", rs)
            meta[f"worst_analytic_over_best_{tag}"] = worst("analytic_ratio", rs)
    save_weights(params, meta, out)
    log(f"[costmodel] test plans, geomean over best: learned {meta['geomean_learned_over_best_all']:.4f}, "
        f"analytic {meta['geomean_analytic_over_best_all']:.4f}; test rmse {test_rmse:.4f}")
    return params, meta


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="measure group times, train the cost network, evaluate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    m = sub.add_parser("measure", help="measure a range of a campaign split into a directory (resumable)")
    m.add_argument("directory")
    m.add_argument("split", choices=["train", "val", "test"])
    m.add_argument("--first", type=int, default=0)
    m.add_argument("--count", type=int, default=None)
    m.add_argument("--reps", type=int, default=3)
    m.add_argument("--max-seconds", type=float, default=None)
    mf = sub.add_parser("measure-fixed", help="measure the fixed-chain campaign (train grid or held-out test)")
    mf.add_argument("directory")
    mf.add_argument("split", choices=["train", "test"])
    mf.add_argument("--reps", type=int, default=5)
    ft = sub.add_parser("finetune", help="fine-tune the shipped network on the fixed-chain tables")
    ft.add_argument("directory")
    ft.add_argument("out", nargs="?", default=WEIGHTS_PATH)
    ft.add_argument("--steps", type=int, default=3000)
    ft.add_argument("--distill-chains", type=int, default=400)
    t = sub.add_parser("train", help="train and evaluate from a directory of tables")
    t.add_argument("directory")
    t.add_argument("out", nargs="?", default=WEIGHTS_PATH)
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--batch", type=int, default=8192)
    a = ap.parse_args()
    say = lambda msg: print(msg, flush=True)
    if a.cmd == "measure":
        complete = measure_cases(a.directory, a.split, a.first, a.count, a.reps, a.max_seconds, log=say)
        say(f"[costmodel] {a.split} measurement {'complete' if complete else 'incomplete'}")
    elif a.cmd == "measure-fixed":
        measure_fixed(a.directory, a.split, a.reps, log=say)
    elif a.cmd == "finetune":
        p0, m0 = load_weights()
        finetune_fixed(a.directory, p0, m0, steps=a.steps, distill_chains=a.distill_chains, out=a.out, log=say)
    else:
        train_from_tables(a.directory, a.steps, a.batch, 5, a.out, log=say)
