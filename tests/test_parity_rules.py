"""CPU checks of the comparison rules the GPU parity tests apply (tests/parity.py).

The wide exemption set is computed sparsely (only pixels that can survive the
threshold have neighbour clauses); here it is compared with the plain dense
statement of the same rule on random response fields with planted
near-threshold values and near-ties.  The literal set is checked on values
placed just inside and just outside 1e-5 of the threshold."""
import numpy as np

from tests import parity


def dense_wide(R, M, thr=parity.THR):
    eps = parity.REL * np.maximum(thr, M)
    near = np.abs(R - thr) <= eps
    p = lambda a: np.pad(a, ((0, 0), (1, 1), (1, 1)), mode="edge")
    Rp, Ep, Np = p(R), p(eps), p(near)
    T, H, W = R.shape
    ex = near.copy()
    live = R >= thr - eps
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            sl = (slice(None), slice(1 + dy, 1 + dy + H), slice(1 + dx, 1 + dx + W))
            rq, eq, nq = Rp[sl], Ep[sl], Np[sl]
            ex |= nq & (rq >= R - eps - eq) & live
            ex |= live & (rq >= thr - eq) & (np.abs(R - rq) <= eps + eq)
    return ex


def planted(seed, shape=(3, 17, 23)):
    rng = np.random.default_rng(seed)
    thr = parity.THR
    R = rng.uniform(-2e8, 4e8, shape)
    M = rng.uniform(0, 3e10, shape)
    flat = R.ravel()
    k = flat.size
    idx = rng.choice(k, k // 6, replace=False)
    flat[idx[: len(idx) // 2]] = thr * (1 + rng.uniform(-3e-5, 3e-5, len(idx) // 2))  # near the threshold
    j = idx[len(idx) // 2:]
    flat[j] = np.roll(flat, 1)[j] * (1 + rng.uniform(-2e-5, 2e-5, len(j)))  # near-ties with a neighbour
    return R, M


def test_sparse_wide_set_equals_dense_statement():
    for seed in range(20):
        R, M = planted(seed)
        wide, _ = parity.decision_sets(R, M)
        assert np.array_equal(wide, dense_wide(R, M)), seed
        assert wide.any()


def test_literal_set():
    thr = parity.THR
    R = np.zeros((1, 5, 5))
    R[0, 2, 2] = thr * (1 + 0.9e-5)   # inside the literal band
    R[0, 0, 0] = thr * (1 + 1.1e-5)   # outside, no literal neighbour
    R[0, 2, 3] = 3 * thr              # survives the threshold next to (2, 2): its decision depends on it
    R[0, 4, 4] = 3 * thr              # survives, no literal neighbour
    M = np.full(R.shape, 1e9)
    wide, lit = parity.decision_sets(R, M)
    assert lit[0, 2, 2] and lit[0, 2, 3]
    assert not lit[0, 0, 0] and not lit[0, 4, 4] and not lit[0, 1, 1]
    # the wide set holds the literal band (eps = 1e-5 M >= 1e-5 thr here)
    assert wide[0, 2, 2] and wide[0, 0, 0]


def test_frame_difference_exemption_covers_the_next_frame():
    ex = np.zeros((3, 2, 2), bool)
    ex[1, 0, 1] = True
    d = parity.diff_exempt(ex)
    assert d[1, 0, 1] and d[2, 0, 1] and not d[0, 0, 1] and d.sum() == 2


def test_point_response_bound():
    pts = np.array([[0, 1, 1, 1.5e8]])
    M = np.full((1, 3, 3), 2e9)  # bound 2e4
    ok = pts.copy()
    ok[0, 3] += 1.9e4
    st = parity.compare_points(ok, pts, np.zeros(M.shape, bool), np.zeros(M.shape, bool), M)
    assert st["points_differ"] == 0 and 0.9 < st["response_err_over_bound"] < 1.0
    bad = pts.copy()
    bad[0, 3] += 2.1e4
    try:
        parity.compare_points(bad, pts, np.zeros(M.shape, bool), np.zeros(M.shape, bool), M)
    except AssertionError:
        pass
    else:
        raise AssertionError("a response error over 1e-5 M was accepted")


def test_generic_full_scale():
    w = np.array([[1, -2, 1]], np.float32)
    assert parity.generic_full_scale([("stencil", 1, 0, w)]) == 255 * 4
    assert parity.generic_full_scale([("box", 1, 2)]) == 255 * 15
    assert parity.generic_full_scale([("point", "affine", -2.0, 5.0)]) == 515
    assert parity.generic_full_scale([("point", "square", 0, 0), ("point", "sqrtabs", 0, 0)]) == 255
    assert parity.generic_full_scale([("point", "clamp", 300.0, 400.0)]) == 300  # every input is below 300
    assert parity.generic_full_scale([("point", "clamp", -10.0, 20.0)]) == 20
    assert abs(parity.north_star_tol([("box", 1, 1)]) - 9e-4) < 1e-15
