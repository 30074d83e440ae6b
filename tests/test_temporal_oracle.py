"""Pins of the oracle's temporal generic stages (no GPU).

IIR filter (Table II, a multi-frame point operation), read as
y[t] = a x[t] + (1 - a) y[t-1] with y[-1] := x[0]; spatio-temporal stencil
(Table I), out(t) = sum_tau w[tau] * in(max(t - tau, 0)), correlated in space
with replicate borders.  Each is checked against something other than
itself: scipy's lfilter (a textbook IIR / FIR routine), closed forms (impulse
and step responses, constants), the frame-by-frame spatial oracle, and brute
force in plain Python on tiny volumes."""
import numpy as np
import pytest
from scipy import signal

import oracle
from paper_1509_04394_amd import synth


def vol(seed, shape=(9, 7, 11)):
    return np.random.default_rng(seed).integers(0, 256, shape).astype(np.float64)


@pytest.mark.parametrize("a", [0.05, 0.3, 0.5, 0.9, 1.0])
def test_iir_equals_lfilter_with_the_first_frame_as_history(a):
    x = vol(int(a * 100))
    y = oracle.gchain([("iir", a)], x)
    # y[n] = a x[n] + (1 - a) y[n-1]: b = [a], den = [1, -(1 - a)]; y[-1] = x[0] is the state zi = (1 - a) x[0]
    ref = signal.lfilter([a], [1.0, -(1.0 - a)], x, axis=0, zi=((1.0 - a) * x[0])[None])[0]
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-9)
    assert np.allclose(y[0], x[0], rtol=1e-15, atol=0)  # y[0] = a x0 + (1 - a) x0, to rounding


def test_iir_closed_forms():
    a, c, t0, T = 0.25, 80.0, 3, 12
    # constant input stays constant
    x = np.full((T, 2, 3), 37.0)
    assert np.allclose(oracle.gchain([("iir", a)], x), 37.0, rtol=0, atol=1e-12)
    # impulse at t0 on a zero background: a c (1 - a)^(t - t0) from t0 on
    x = np.zeros((T, 2, 3))
    x[t0] = c
    y = oracle.gchain([("iir", a)], x)
    want = np.array([0.0 if t < t0 else a * c * (1 - a) ** (t - t0) for t in range(T)])
    assert np.allclose(y[:, 1, 2], want, rtol=1e-13, atol=1e-13)
    # step at t0: c (1 - (1 - a)^(t - t0 + 1))
    x = np.zeros((T, 2, 3))
    x[t0:] = c
    y = oracle.gchain([("iir", a)], x)
    want = np.array([0.0 if t < t0 else c * (1 - (1 - a) ** (t - t0 + 1)) for t in range(T)])
    assert np.allclose(y[:, 0, 0], want, rtol=1e-13, atol=1e-12)
    # a = 1 is the identity
    x = vol(5)
    assert np.array_equal(oracle.gchain([("iir", 1.0)], x), x)


def test_temporal_stencil_with_one_frame_is_the_spatial_stencil():
    x = vol(7)
    w = np.random.default_rng(8).standard_normal((3, 5))
    a = oracle.gchain([("stencil", 2, 1, w[None])], x)
    b = oracle.gchain([("stencil", 2, 1, w)], x)  # frame-by-frame spatial oracle
    assert np.allclose(a, b, rtol=1e-13, atol=1e-10)


def test_temporal_fir_equals_lfilter_with_replicated_first_frame():
    x = vol(9, (10, 3, 4))
    om = np.array([0.5, -0.25, 0.125, 2.0])
    w = om.reshape(4, 1, 1)
    y = oracle.gchain([("stencil", 0, 0, w)], x)
    pad = np.concatenate([np.repeat(x[:1], 3, axis=0), x])  # frames before the first are the first
    ref = signal.lfilter(om, [1.0], pad, axis=0)[3:]
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-10)


def test_separable_space_time_stencil():
    x = vol(11, (6, 8, 9))
    om = np.array([0.6, 0.3, 0.1])
    k = np.random.default_rng(12).standard_normal((3, 3))
    y = oracle.gchain([("stencil", 1, 1, om[:, None, None] * k[None])], x)
    sp = oracle.gchain([("stencil", 1, 1, k)], x)
    ref = sum(om[tau] * sp[np.maximum(np.arange(6) - tau, 0)] for tau in range(3))
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-10)


def brute(stages, x):
    """Plain-Python loops over every pixel of every stage (tiny volumes only)."""
    T, H, W = x.shape
    cl = lambda v, n: min(max(v, 0), n - 1)
    cur = x.tolist()
    for st in stages:
        nxt = [[[0.0] * W for _ in range(H)] for _ in range(T)]
        if st[0] == "iir":
            a = st[1]
            for yy in range(H):
                for xx in range(W):
                    prev = cur[0][yy][xx]
                    for t in range(T):
                        prev = a * cur[t][yy][xx] + (1 - a) * prev
                        nxt[t][yy][xx] = prev
        elif st[0] == "stencil":
            w = np.asarray(st[3], np.float64)
            w = w if w.ndim == 3 else w[None]
            rx, ry = st[1], st[2]
            for t in range(T):
                for yy in range(H):
                    for xx in range(W):
                        acc = 0.0
                        for tau in range(w.shape[0]):
                            for v in range(-ry, ry + 1):
                                for u in range(-rx, rx + 1):
                                    acc += w[tau, v + ry, u + rx] * cur[max(t - tau, 0)][cl(yy + v, H)][cl(xx + u, W)]
                        nxt[t][yy][xx] = acc
        elif st[0] == "point" and st[1] == "abs":
            nxt = [[[abs(v) for v in row] for row in fr] for fr in cur]
        cur = nxt
    return np.array(cur)


def test_brute_force_chains_on_tiny_volumes():
    rng = np.random.default_rng(13)
    x = rng.integers(0, 256, (5, 4, 6)).astype(np.float64)
    w3 = rng.standard_normal((3, 3, 5))  # rt = 2, ry = 1, rx = 2
    for stages in ([("iir", 0.4), ("stencil", 2, 1, w3)],
                   [("stencil", 2, 1, w3), ("point", "abs", 0, 0), ("iir", 0.7)],
                   [("iir", 0.3), ("iir", 0.6)]):
        assert np.allclose(oracle.gchain(stages, x), brute(stages, x), rtol=1e-12, atol=1e-9), stages


def test_stage_major_equals_frame_major_without_time(monkeypatch):
    """The stage-by-stage driver gives the frame-by-frame driver's result on
    chains without a temporal stage (the same stage routines, in another
    loop order)."""
    for seed in (5000, 5003, 5006):
        spec = synth.random_chain(seed, length=6)
        x = synth.video(40, 30, 3, seed=seed).astype(np.float64)
        frame_major = oracle.gchain(spec, x)
        monkeypatch.setattr(oracle, "_temporal", lambda st: True)
        stage_major = oracle.gchain(spec, x)
        monkeypatch.undo()
        assert np.array_equal(frame_major, stage_major), seed
