"""Pins of the oracle's generic stages (point, weighted stencil, window sum).

These are the Table I access classes with free parameters.  Each stage is
checked against a library routine that computes the same definition
(``scipy.ndimage.correlate`` / ``uniform_filter`` with mode 'nearest' =
replicate borders, numpy's elementwise functions), against closed forms
(ramps, constants, linearity), and against brute force on frames smaller
than the window.  Mistakes these catch: convolution instead of correlation
(a flipped or transposed weight array: asymmetric weights with rx != ry),
a wrong border rule (tiny frames), a dropped row or column of the window
(library match), a wrong point formula or parameter order, stages applied out
of order, or frames mixed up.
"""
import numpy as np
import pytest
from scipy import ndimage

from paper_1509_04394_amd import synth


def _frames(shape, seed, lo=0, hi=256):
    return np.random.default_rng(seed).integers(lo, hi, shape).astype(np.float64)


@pytest.mark.parametrize("rx,ry,shape", [(2, 1, (2, 9, 11)), (0, 3, (1, 12, 7)), (3, 3, (1, 4, 3)),
                                         (1, 0, (3, 5, 40))])
def test_stencil_matches_scipy_correlate(oracle_lib, rx, ry, shape):
    rng = np.random.default_rng(rx * 10 + ry)
    w = rng.standard_normal((2 * ry + 1, 2 * rx + 1))
    v = _frames(shape, 3)
    out = oracle_lib.gchain([("stencil", rx, ry, w)], v)
    for t in range(shape[0]):
        ref = ndimage.correlate(v[t], w, mode="nearest")
        np.testing.assert_allclose(out[t], ref, rtol=1e-12, atol=1e-9)


def test_stencil_orientation_on_a_ramp(oracle_lib):
    # w multiplies in(x+u, y+v) at w[v+ry][u+rx]: a forward difference along x
    # on the ramp 3x + 5y gives +3 inside the frame and 0 at the right edge.
    W, H = 9, 6
    ramp = (3.0 * np.arange(W)[None, :] + 5.0 * np.arange(H)[:, None])[None]
    wx = np.zeros((3, 3))
    wx[1, 1], wx[1, 2] = -1.0, 1.0
    out = oracle_lib.gchain([("stencil", 1, 1, wx)], ramp)[0]
    assert np.all(out[:, :-1] == 3.0) and np.all(out[:, -1] == 0.0)
    wy = np.zeros((5, 1))
    wy[2, 0], wy[4, 0] = -1.0, 1.0  # rx = 0, ry = 2: in(x, y+2) - in(x, y)
    out = oracle_lib.gchain([("stencil", 0, 2, wy)], ramp)[0]
    assert np.all(out[: H - 2] == 10.0)
    assert np.all(out[H - 2] == 5.0) and np.all(out[H - 1] == 0.0)


def test_stencil_invariants(oracle_lib):
    rng = np.random.default_rng(7)
    v = _frames((2, 10, 13), 8)
    delta = np.zeros((5, 7))
    delta[2, 3] = 1.0
    assert np.array_equal(oracle_lib.gchain([("stencil", 3, 2, delta)], v), v)
    w = rng.standard_normal((3, 5))
    c = np.full((1, 6, 6), 17.0)
    np.testing.assert_allclose(oracle_lib.gchain([("stencil", 2, 1, w)], c), 17.0 * w.sum(), rtol=1e-12)
    a, b = _frames((1, 8, 9), 9), _frames((1, 8, 9), 10)
    lhs = oracle_lib.gchain([("stencil", 2, 1, w)], 2.0 * a - 3.0 * b)
    rhs = 2.0 * oracle_lib.gchain([("stencil", 2, 1, w)], a) - 3.0 * oracle_lib.gchain([("stencil", 2, 1, w)], b)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("rx,ry,shape", [(1, 1, (2, 8, 9)), (3, 1, (1, 10, 12)), (2, 3, (1, 5, 4))])
def test_box_matches_uniform_filter(oracle_lib, rx, ry, shape):
    v = _frames(shape, 11)
    out = oracle_lib.gchain([("box", rx, ry)], v)
    area = (2 * rx + 1) * (2 * ry + 1)
    for t in range(shape[0]):
        ref = ndimage.uniform_filter(v[t], size=(2 * ry + 1, 2 * rx + 1), mode="nearest") * area
        np.testing.assert_allclose(out[t], ref, rtol=1e-12, atol=1e-8)


def test_box_brute_force_on_a_frame_smaller_than_the_window(oracle_lib):
    v = np.array([[[1.0, 2.0, 4.0], [8.0, 16.0, 32.0]]])  # H = 2, W = 3, window 7 x 7
    out = oracle_lib.gchain([("box", 3, 3)], v)[0]
    for y in range(2):
        for x in range(3):
            # a replicate-bordered 7 x 7 window counts every pixel by how many
            # clamped offsets land on it
            cnt_x = [sum(1 for u in range(-3, 4) if min(max(x + u, 0), 2) == i) for i in range(3)]
            cnt_y = [sum(1 for u in range(-3, 4) if min(max(y + u, 0), 1) == j) for j in range(2)]
            ref = sum(cnt_y[j] * cnt_x[i] * v[0, j, i] for j in range(2) for i in range(3))
            assert out[y, x] == ref


def test_point_ops_match_numpy(oracle_lib):
    v = np.random.default_rng(12).uniform(-300, 300, (2, 7, 9))
    cases = {
        ("point", "affine", -1.5, 7.25): -1.5 * v + 7.25,
        ("point", "abs", 0.0, 0.0): np.abs(v),
        ("point", "square", 0.0, 0.0): np.square(v),
        ("point", "sqrtabs", 0.0, 0.0): np.sqrt(np.abs(v)),
        ("point", "clamp", -20.0, 55.5): np.clip(v, -20.0, 55.5),
    }
    for st, ref in cases.items():
        np.testing.assert_allclose(oracle_lib.gchain([st], v), ref, rtol=1e-15, atol=0, err_msg=str(st))


def test_chain_composes_in_order_frame_by_frame(oracle_lib):
    rng = np.random.default_rng(13)
    w = rng.standard_normal((5, 3))
    stages = [("point", "affine", 0.5, -10.0), ("stencil", 1, 2, w), ("point", "abs", 0, 0), ("box", 2, 1),
              ("point", "sqrtabs", 0, 0), ("point", "clamp", 1.0, 9.0)]
    v = _frames((4, 11, 14), 14)
    out = oracle_lib.gchain(stages, v)
    for t in range(4):
        x = 0.5 * v[t] - 10.0
        x = np.abs(ndimage.correlate(x, w, mode="nearest"))
        x = ndimage.uniform_filter(x, size=(3, 5), mode="nearest") * 15
        x = np.clip(np.sqrt(np.abs(x)), 1.0, 9.0)
        np.testing.assert_allclose(out[t], x, rtol=1e-12, atol=1e-12)
    # frames are independent: permuting them permutes the output
    perm = [2, 0, 3, 1]
    np.testing.assert_array_equal(oracle_lib.gchain(stages, v[perm]), out[perm])


def test_random_chain_recipe():
    a, b = synth.random_chain(5001), synth.random_chain(5001)
    assert len(a) == len(b) and 4 <= len(a) <= 16
    for sa, sb in zip(a, b):
        assert sa[0] == sb[0]
        if sa[0] == "stencil":
            assert sa[1] == sa[2] and 0 <= sa[1] <= 3
            assert sa[3].dtype == np.float32 and np.array_equal(sa[3], sb[3])
            assert abs(float(np.abs(sa[3].astype(np.float64)).sum()) - 1.0) < 1e-5
        elif sa[0] == "box":
            assert 1 <= sa[1] == sa[2] <= 3
        else:
            assert sa == sb and sa[1] in synth.POINT_KINDS
            if sa[1] == "clamp":
                assert sa[2] < sa[3]
    kinds = {s[0] for k in range(40) for s in synth.random_chain(k)}
    assert kinds == {"stencil", "point", "box"}
