"""Pins of the tracking oracle (oracle/track.c): the Kalman filter with a
constant-velocity model and greedy nearest-neighbour association that the
paper's pipeline applies to its feature points (Sec. III, Table II).

Independent checks: a stationary point is held exactly; a noise-free
constant-velocity target is followed, and the oracle's states equal a plain
numpy matrix implementation of the textbook filter (np.linalg.inv for S^-1)
to 1e-9; that implementation's predicted covariance converges to the
discrete algebraic Riccati equation's solution from scipy; hand-built frames
fix the association order (ties by track id), the drop after max_miss missed
frames and the order of new ids."""
import numpy as np
import pytest

import oracle


def recs(points, T, **kw):
    ints, st = oracle.track(np.array(points, np.int64).reshape(-1, 3), T, **kw)
    return [tuple(int(v) for v in a) + tuple(float(v) for v in b) for a, b in zip(ints, st)]


def test_empty_input_gives_no_tracks():
    ints, st = oracle.track(np.zeros((0, 3), np.int64), 10)
    assert len(ints) == 0 and len(st) == 0


def test_stationary_point_is_held_exactly():
    T = 12
    pts = [(t, 40, 25) for t in range(T)]
    r = recs(pts, T)
    assert len(r) == T
    assert r[0][:3] == (0, 0, 2)
    for t, rec in enumerate(r):
        assert rec[:2] == (t, 0) and rec[2] == (2 if t == 0 else 1)
        assert rec[3:] == (25.0, 40.0, 0.0, 0.0)


def kalman_numpy(zs, q, r, v0):
    """The textbook filter in matrix form (independent of the oracle's
    summation order): returns the states after each frame and the predicted
    covariances."""
    F = np.array([[1, 0, 1, 0], [0, 1, 0, 1], [0, 0, 1, 0], [0, 0, 0, 1]], float)
    Q = q * np.array([[.25, 0, .5, 0], [0, .25, 0, .5], [.5, 0, 1, 0], [0, .5, 0, 1]])
    H = np.array([[1, 0, 0, 0], [0, 1, 0, 0]], float)
    R = r * np.eye(2)
    s = np.array([zs[0][0], zs[0][1], 0, 0], float)
    P = np.diag([r, r, v0, v0])
    out, Ppred = [s.copy()], []
    for z in zs[1:]:
        s = F @ s
        P = F @ P @ F.T + Q
        Ppred.append(P.copy())
        S = H @ P @ H.T + R
        K = P @ H.T @ np.linalg.inv(S)
        s = s + K @ (np.asarray(z, float) - H @ s)
        P = (np.eye(4) - K @ H) @ P
        out.append(s.copy())
    return np.array(out), Ppred, (F, Q, H, R)


def test_constant_velocity_target_matches_matrix_form_and_converges():
    T, vx, vy = 60, 2, -1
    pts = [(t, 300 + vy * t, 10 + vx * t) for t in range(T)]
    r = recs(pts, T)
    assert [x[1] for x in r] == [0] * T  # one track throughout
    got = np.array([x[3:] for x in r])
    zs = [(10 + vx * t, 300 + vy * t) for t in range(T)]
    ref, Ppred, (F, Q, H, R) = kalman_numpy(zs, 0.5, 1.0, 4.0)
    assert np.allclose(got, ref, rtol=0, atol=1e-9)
    # the filter follows the target: position exact to 1e-6, velocity to 1e-6 by the end
    assert abs(got[-1, 0] - zs[-1][0]) < 1e-6 and abs(got[-1, 1] - zs[-1][1]) < 1e-6
    assert abs(got[-1, 2] - vx) < 1e-6 and abs(got[-1, 3] - vy) < 1e-6
    # predicted covariance -> the discrete algebraic Riccati solution
    from scipy.linalg import solve_discrete_are
    X = solve_discrete_are(F.T, H.T, Q, R)
    assert np.allclose(Ppred[-1], X, rtol=1e-8, atol=1e-10)


def test_random_walk_targets_match_matrix_form():
    """Three well separated targets with random integer jitter: one track
    each, states equal to the matrix form per target."""
    rng = np.random.default_rng(5)
    T = 40
    starts = [(20, 30), (200, 40), (110, 300)]
    paths = []
    for (x0, y0) in starts:
        v = rng.integers(-2, 3, size=2)
        p = [(int(x0 + v[0] * t + rng.integers(-1, 2)), int(y0 + v[1] * t + rng.integers(-1, 2))) for t in range(T)]
        paths.append(p)
    pts = [(t, p[t][1], p[t][0]) for t in range(T) for p in paths]
    r = recs(pts, T)
    by_id = {}
    for rec in r:
        by_id.setdefault(rec[1], []).append(rec)
    assert len(by_id) == 3
    for k, p in enumerate(sorted(paths, key=lambda p: (p[0][1], p[0][0]))):
        got = np.array([x[3:] for x in by_id[k]])
        ref, _, _ = kalman_numpy(p, 0.5, 1.0, 4.0)
        assert np.allclose(got, ref, rtol=0, atol=1e-9)


def test_association_order_ties_by_track_id():
    """Frame 0: tracks 0 at x=10 and 1 at x=14.  Frame 1: points at x=12 and
    x=16.  Both tracks see x=12 at the same distance (identical covariances):
    the lower id takes it, track 1 takes x=16."""
    pts = [(0, 10, 10), (0, 10, 14), (1, 10, 12), (1, 10, 16)]
    r = recs(pts, 2, gate=100.0)
    f1 = {x[1]: x for x in r if x[0] == 1}
    assert f1[0][2] == 1 and f1[1][2] == 1
    # the update moves each track toward its point: track 0 right of 10, track 1 right of 14
    assert 10 < f1[0][3] < 12 and 14 < f1[1][3] < 16
    # swap the point order in the input: same result (points are ordered by (y, x))
    r2 = recs([pts[1], pts[0], pts[3], pts[2]], 2, gate=100.0)
    assert r2 == r


def test_gate_drop_and_new_ids():
    """A point seen in frames 0-4 then gone: its track is predicted for
    max_miss frames (status 0) and dropped; a far point starts a new track
    (the gate keeps it from the old one); new ids follow (y, x) order."""
    mm = 2
    pts = [(t, 50, 50) for t in range(5)] + [(6, 200, 5), (6, 100, 300), (6, 100, 20)]
    r = recs(pts, 10, max_miss=mm)
    t0 = [x for x in r if x[1] == 0]
    assert [x[0] for x in t0] == list(range(5 + mm))
    assert [x[2] for x in t0[5:]] == [0] * mm
    born = sorted((x[1], x[3], x[4]) for x in r if x[2] == 2 and x[0] == 6)
    # ids 1, 2, 3 in (y, x) order: (100, 20), (100, 300), (200, 5)
    assert [(b[1], b[2]) for b in born] == [(20.0, 100.0), (300.0, 100.0), (5.0, 200.0)]
    assert [b[0] for b in born] == [1, 2, 3]


def test_greedy_is_not_optimal_assignment():
    """Greedy nearest neighbour (the stated rule), not the least total
    distance: tracks 0 at x=10 and 1 at x=13, points at x=12 and x=15 (gate
    open).  Track 1 is closest to x=12 (distance 1) and takes it first, so
    track 0 gets x=15 (distance 5): total 6, where pairing 0-12 and 1-15
    would cost 2 + 2."""
    pts = [(0, 20, 10), (0, 20, 13), (1, 20, 12), (1, 20, 15)]
    r = recs(pts, 2, gate=1e9)
    f1 = {x[1]: x for x in r if x[0] == 1}
    assert f1[0][2] == 1 and f1[1][2] == 1
    assert 10 < f1[0][3] < 15  # track 0 pulled right, toward x=15
    assert 12 < f1[1][3] < 13  # track 1 pulled left, toward x=12
