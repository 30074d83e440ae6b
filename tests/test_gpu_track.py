"""GPU parity of the tracking stage (fz_track_points) against the oracle.

The stage the paper applies after the chain (Sec. III; Table II's Kalman
filter, Table IV's kernel-to-kernel dependent K6) runs on the point list the
chain's suppression stage wrote.  Both sides evaluate the same double-
precision sums in the same order, so every record -- frame, track id,
status and the four state values -- must be equal to the bit: the
association is index work."""
import numpy as np
import pytest

import oracle
from paper_1509_04394_amd import fz, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-track]", *a, flush=True)


@pytest.fixture(scope="module")
def dev(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_points(rows, dev, cap=None):
    """A point buffer as the chain writes it: (cap, 4) int32 rows (t, y, x,
    response bits) and the count."""
    rows = np.asarray(rows, np.int64).reshape(-1, 3)
    cap = cap or max(len(rows), 1)
    buf = np.zeros((cap, 4), np.int32)
    buf[:len(rows), :3] = rows
    return (torch.from_numpy(buf).to(dev), torch.tensor([len(rows)], dtype=torch.int32, device=dev))


def compare(rec, flags, pts_tyx, T, **kw):
    assert flags == 0, flags
    oi, od = oracle.track(pts_tyx, T, **kw)
    g = sorted((int(r["t"]), int(r["id"]), int(r["status"]), float(r["x"]), float(r["y"]), float(r["vx"]),
                float(r["vy"])) for r in rec)
    o = sorted((int(a[0]), int(a[1]), int(a[2])) + tuple(float(v) for v in b) for a, b in zip(oi, od))
    assert len(g) == len(o), (len(g), len(o))
    bad = [(x, y) for x, y in zip(g, o) if x != y]
    assert not bad, f"{len(bad)} records differ, first {bad[:3]}"
    return len(g)


def test_hand_made_point_lists(dev):
    cases = [
        ([(t, 40, 25) for t in range(12)], 12, {}),
        ([(0, 10, 10), (0, 10, 14), (1, 10, 12), (1, 10, 16)], 2, dict(gate=100.0)),
        ([(0, 20, 10), (0, 20, 13), (1, 20, 12), (1, 20, 15)], 2, dict(gate=1e9)),
        ([(t, 50, 50) for t in range(5)] + [(6, 200, 5), (6, 100, 300), (6, 100, 20)], 10, dict(max_miss=2)),
        ([(t, 300 - t, 10 + 2 * t) for t in range(60)], 60, {}),
    ]
    for rows, T, kw in cases:
        pts, cnt = gpu_points(rows, dev)
        o = fz.track_opts(**kw)
        rec, flags = fz.track_points(pts, cnt, T, o)
        n = compare(rec, flags, np.array(rows), T, **kw)
        say("hand-made", len(rows), "points", n, "records")


def test_empty_and_out_of_range_points(dev):
    pts, cnt = gpu_points([], dev, cap=8)
    rec, flags = fz.track_points(pts, cnt, 5)
    assert len(rec) == 0 and flags == 0
    # points beyond the clip's frames are ignored
    pts, cnt = gpu_points([(0, 5, 5), (1, 5, 6), (9, 5, 7)], dev)
    rec, flags = fz.track_points(pts, cnt, 3)
    compare(rec, flags, np.array([(0, 5, 5), (1, 5, 6)]), 3)


def test_chain_points_tracked(dev):
    """The Harris chain's points on synthetic video (20 moving blobs), then
    the tracker, against the oracle tracking the same points."""
    for (W, H, T, seed) in [(192, 432, 60, 2), (320, 240, 97, 9)]:
        vol = synth.video(W, H, T, seed=seed)
        plan = fz.Plan(fz.HARRIS_CHAIN, W, H, T)
        x = torch.from_numpy(vol).to(dev)
        out, pts, cnt = plan.run(x)
        torch.cuda.synchronize()
        n_pts = int(cnt.item())
        rec, flags = fz.track_points(pts, cnt, T)
        host = pts[:n_pts, :3].cpu().numpy()
        n = compare(rec, flags, host, T)
        say(f"{W}x{H}x{T}: {n_pts} points, {n} track records, {len(set(rec['id'].tolist()))} tracks")


def test_dense_frames_and_wide_coordinates(dev):
    """Frames past one wavefront's registers: 144 points a frame (the sort
    through LDS), 144 live tracks (tracks past the first 64 in the
    workspace) and over a thousand gated candidates (association rounds
    reading candidates from LDS), on a jittered grid drifting right and
    down; frames above and below 64 points in turn; then points with
    negative and 17-bit coordinates (the (y, x) order of the sort as signed
    integers)."""
    rng = np.random.default_rng(11)
    rows = []
    for t in range(10):
        for gy in range(12):
            for gx in range(12):
                rows.append((t, 20 + 4 * gy + t // 2 + int(rng.integers(-1, 2)), 30 + 4 * gx + t + int(rng.integers(-1, 2))))
    rows = list({r: None for r in rows})  # (t, y, x) keys distinct within a frame
    pts, cnt = gpu_points(rows, dev)
    rec, flags = fz.track_points(pts, cnt, 10)
    n = compare(rec, flags, np.array(rows), 10)
    say("dense grid", len(rows), "points", n, "records")
    # frames above and below 64 points in turn (a frame of at most 64 is sorted
    # while the one before it is associated, a larger one at its own start)
    rows = []
    for t, n in enumerate([30, 100, 20, 70, 64, 65, 10, 90, 64, 1]):
        cells = rng.choice(16 * 16, size=n, replace=False)
        rows += [(t, 30 + 5 * int(c // 16) + t, 40 + 5 * int(c % 16) + t // 2) for c in cells]
    pts, cnt = gpu_points(rows, dev)
    rec, flags = fz.track_points(pts, cnt, 10)
    n = compare(rec, flags, np.array(rows), 10)
    say("mixed frame sizes", len(rows), "points", n, "records")
    rows = [(0, -5, 3), (0, -5, -2), (0, 70000, 1), (0, 2, 70000), (0, -70000, 9),
            (1, -4, 3), (1, 70001, 2), (1, 3, 69999), (1, -69999, 8), (2, -3, 4)]
    pts, cnt = gpu_points(rows, dev)
    rec, flags = fz.track_points(pts, cnt, 3)
    n = compare(rec, flags, np.array(rows), 3)
    say("wide coordinates", n, "records")


def test_limits_are_flagged(dev):
    # a frame with more points than one wavefront's frame buffer holds (1024)
    rows = [(0, y, x) for y in range(0, 66, 2) for x in range(0, 66, 2)]  # 1089 points
    pts, cnt = gpu_points(rows, dev)
    _, flags = fz.track_points(pts, cnt, 1)
    assert flags & fz.FZ_TRACK_TOO_MANY_POINTS
    # more gated pairs in a frame than the list holds (2048): 60 tracks, each
    # gating all 60 points of the next frame
    rows = [(t, 10 + 3 * (k // 8), 10 + 3 * (k % 8)) for t in range(2) for k in range(60)]
    pts, cnt = gpu_points(rows, dev)
    _, flags = fz.track_points(pts, cnt, 2, fz.track_opts(gate=1e9))
    assert flags & fz.FZ_TRACK_TOO_MANY_CANDIDATES
    # more live tracks than allowed
    rows = [(0, 10 * k, 10 * k) for k in range(8)]
    pts, cnt = gpu_points(rows, dev)
    rec, flags = fz.track_points(pts, cnt, 1, fz.track_opts(max_tracks=3))
    assert flags & fz.FZ_TRACK_TOO_MANY_TRACKS and len(rec) == 3


def test_bad_arguments_are_refused(dev):
    pts, cnt = gpu_points([(0, 1, 1)], dev)
    for kw in (dict(r=0.0), dict(q=-1.0), dict(max_tracks=0), dict(max_tracks=5000), dict(max_miss=-1)):
        with pytest.raises(fz.FzError):
            fz.track_points(pts, cnt, 3, fz.track_opts(**kw))
    with pytest.raises(fz.FzError):
        fz.track_points(pts, cnt, 0)


def test_full_size_workload_points_tracked(dev):
    """The 800x600x1000 RGB workload's points (the benchmark's chain), all
    1000 frames tracked, against the oracle."""
    W, H, T = 800, 600, 1000
    rgb = synth.video(W, H, T, seed=3, rgb=True)
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T)
    x = torch.from_numpy(rgb).to(dev)
    del rgb
    out, pts, cnt = plan.run(x)
    torch.cuda.synchronize()
    del x, out
    n_pts = int(cnt.item())
    rec, flags = fz.track_points(pts, cnt, T)
    n = compare(rec, flags, pts[:n_pts, :3].cpu().numpy(), T)
    say(f"800x600x1000: {n_pts} points, {n} records, {len(set(rec['id'].tolist()))} tracks")
