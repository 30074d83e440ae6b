"""Pins of the brute-force partition oracle (Sec. VI, Fig. 5 model)."""
import math

import pytest

from oracle import partition as P


def test_three_kernels_have_four_partitions():
    # Sec. VI lists exactly these four for K1, K2, K3
    got = sorted(P.partitions(3))
    want = sorted([[(0, 0), (1, 1), (2, 2)], [(0, 2)], [(0, 1), (2, 2)], [(0, 0), (1, 2)]])
    assert got == want


@pytest.mark.parametrize("n", range(1, 11))
def test_counts(n):
    assert P.n_partitions(n) == 2 ** (n - 1)
    assert P.n_candidates(n) == n * (n + 1) // 2  # Fig. 5
    for groups in P.partitions(n):  # exact cover, in order
        covered = [i for a, b in groups for i in range(a, b + 1)]
        assert covered == list(range(n))


def test_hand_worked_optimum():
    inf = math.inf
    # 4 kernels; fusing 0..1 is cheap, 2 cannot join anything, 3 alone is cheap
    c = [[10, 4, inf, inf], [None, 10, inf, inf], [None, None, 3, inf], [None, None, None, 2]]
    total, groups = P.best(c, 4)
    assert total == 9 and groups == [(0, 1), (2, 2), (3, 3)]


def test_tie_rule_fewer_groups_then_late_cuts():
    # every partition of 3 costs the same -> the single group wins
    c = [[3, 2, 1], [None, 1, 0], [None, None, 1]]
    c[0][2] = 3
    total, groups = P.best(c, 3)
    assert total == 3 and groups == [(0, 2)]
    # two two-group partitions tie: cut after 1 is later than cut after 0
    c = [[1, 2, 9], [None, 5, 2], [None, None, 1]]
    total, groups = P.best(c, 3)
    assert total == 3 and groups == [(0, 1), (2, 2)]


def test_infeasible_everything():
    inf = math.inf
    c = [[inf, inf], [None, inf]]
    total, _ = P.best(c, 2)
    assert math.isinf(total)


def test_traffic_model_eq1_eq2():
    # bytes in/out per pixel of a three-kernel chain u8 -> f32 -> 2xf32 -> f32
    bi, bo = [1, 4, 8], [4, 8, 4]
    assert P.unfused_bytes(bi, bo) == 29  # Eq. 1: every kernel reads and writes
    assert P.compulsory_bytes(bi, bo, 0, 2) == 5  # Eq. 2: one read, one write
    assert P.compulsory_bytes(bi, bo, 1, 1) == 12
    assert P.compulsory_bytes([1], [1], 0, 0, temporal_reread=[0.25]) == 2.25
