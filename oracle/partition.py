"""Brute-force partition oracle -- TEST INFRASTRUCTURE ONLY.

Sec. VI (Fig. 5): a fusable set of n kernels in a fixed order is split into
contiguous groups, each group becoming one fused kernel; the chosen groups must
cover every kernel exactly once, and the total predicted cost of the chosen
groups is minimised.  With three kernels there are four such partitions, and a
set of n kernels offers n(n+1)/2 candidate groups (the contiguous runs).

This module enumerates every one of the 2^(n-1) partitions (one bit per gap
between neighbouring kernels) and scores it, which is the definition of the
optimum; the GPU library solves the same model by dynamic programming.

Tie rule where several partitions share the minimum cost (the paper does not
say): fewer groups first, then the partition whose sorted cut list is
lexicographically larger (cuts as late as possible).
"""
from __future__ import annotations

import itertools


def partitions(n: int):
    """Yield every partition of kernels 0..n-1 into contiguous groups, each as a
    list of (first, last) index pairs."""
    if n <= 0:
        return
    for bits in itertools.product((0, 1), repeat=n - 1):
        groups, start = [], 0
        for gap, cut in enumerate(bits):
            if cut:
                groups.append((start, gap))
                start = gap + 1
        groups.append((start, n - 1))
        yield groups


def candidate_groups(n: int):
    """The n(n+1)/2 contiguous runs a fused kernel may cover."""
    return [(a, b) for a in range(n) for b in range(a, n)]


def cuts_of(groups):
    """Last-kernel index of every group but the final one."""
    return [b for (_, b) in groups[:-1]]


def best(cost, n: int):
    """Exhaustive optimum of the Fig. 5 model.

    ``cost[a][b]`` is the cost of fusing kernels a..b into one kernel
    (``math.inf`` if that group is not allowed).  Returns (total, groups); total
    is inf when no partition is feasible.
    """
    best_key, best_groups = None, None
    for groups in partitions(n):
        total = 0.0
        for a, b in groups:
            total += cost[a][b]
        key = (total, len(groups), [-c for c in cuts_of(groups)])
        if best_key is None or key < best_key:
            best_key, best_groups = key, groups
    return best_key[0], best_groups


def compulsory_bytes(bytes_in, bytes_out, a: int, b: int, temporal_reread=None) -> float:
    """Bytes per pixel moved between global memory and the chip by one fused
    kernel covering kernels a..b (Eq. 2: one access of the group's input, one
    write of its output).  ``temporal_reread[s]`` adds the extra input fraction a
    multi-frame kernel s re-reads."""
    extra = 0.0
    if temporal_reread is not None:
        extra = sum(temporal_reread[s] for s in range(a, b + 1))
    return bytes_in[a] + bytes_out[b] + extra


def unfused_bytes(bytes_in, bytes_out) -> float:
    """Eq. 1 traffic of the plain sequence: every kernel reads its input and
    writes its output."""
    return float(sum(bytes_in) + sum(bytes_out))


def n_partitions(n: int) -> int:
    return sum(1 for _ in partitions(n))


def n_candidates(n: int) -> int:
    return len(candidate_groups(n))

