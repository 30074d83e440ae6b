"""Comparison rules between the GPU library and the FP64 oracle.

Floating-point stages: |gpu - oracle| <= 1e-4 on a 0-255 scale, i.e. 1e-4 of
the stage's full-scale value for uint8 input divided by 255:
  gauss 255, sobel 4*255, gradmag sqrt(2)*4*255, products (4*255)^2,
  box sums 25*(4*255)^2, harris / threshold (25*(4*255)^2)^2.

Integer outputs (gray, mask, frame difference) and feature points are compared
exactly, except at pixels whose decision FP32 rounding can flip: the response
R is compared with the threshold and with its neighbours, and FP32 evaluates
R = Sxx*Syy - Sxy^2 - k (Sxx+Syy)^2 with an error proportional to the size of
its terms, M = |Sxx*Syy| + Sxy^2 + k (Sxx+Syy)^2, not to R.  A pixel is exempt
when its response lies within eps = 1e-5 * max(thr, M) of the threshold, or
within eps of a neighbour's response that could beat it.  The exempt set is
reported and expected to be (nearly) empty.
"""
from __future__ import annotations

import numpy as np

FULL_SCALE = {
    "gauss5": 255.0,
    "sobel3": 1020.0,
    "gradmag": 1020.0 * np.sqrt(2.0),
    "products": 1020.0 ** 2,
    "boxsum5": 25 * 1020.0 ** 2,
    "harris": (25 * 1020.0 ** 2) ** 2,
    "threshold": (25 * 1020.0 ** 2) ** 2,
}
THR = 1.0e8
K = 0.04
REL = 1e-5


def fp_tol(op: str) -> float:
    return 1e-4 * FULL_SCALE[op] / 255.0


def term_size(S):
    """M per pixel from window sums S = (Sxx, Sxy, Syy) [3][T][H][W]."""
    sxx, sxy, syy = S
    return np.abs(sxx * syy) + sxy * sxy + K * (sxx + syy) ** 2


def neighbours(a, fill_edge=True):
    """The 8 replicate-border 3x3 neighbours of every pixel of a [T][H][W] array."""
    p = np.pad(a, ((0, 0), (1, 1), (1, 1)), mode="edge")
    T, H, W = a.shape
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            out.append(p[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W])
    return out


def decision_exempt(R, M, thr=THR):
    """Boolean [T][H][W]: pixels whose suppression mask FP32 may legitimately flip."""
    eps = REL * np.maximum(thr, M)
    near_thr = np.abs(R - thr) <= eps
    ex = near_thr.copy()
    Rn, En, Tn = neighbours(R), neighbours(eps), neighbours(near_thr)
    live = R >= thr - eps
    for rq, eq, tq in zip(Rn, En, Tn):
        # a neighbour whose survival is uncertain and that may beat this pixel
        ex |= tq & (rq >= R - eps - eq) & live
        # a near-tie between two surviving responses
        ex |= live & (rq >= thr - eq) & (np.abs(R - rq) <= eps + eq)
    return ex


def diff_exempt(mask_exempt):
    """Frame-difference pixels that depend on an exempt mask pixel (t or t-1)."""
    ex = mask_exempt.copy()
    ex[1:] |= mask_exempt[:-1]
    return ex


def point_key(pts):
    return {(int(p[0]), int(p[1]), int(p[2])) for p in pts}


def compare_points(gpu, ora, exempt, tol_r):
    """Point sets equal outside exempt pixels; responses within tol_r."""
    g = {k: r for k, r in zip(map(tuple, gpu[:, :3].astype(int).tolist()), gpu[:, 3])}
    o = {k: r for k, r in zip(map(tuple, ora[:, :3].astype(int).tolist()), ora[:, 3])}
    bad = []
    for k in set(g) ^ set(o):
        if not exempt[k]:
            bad.append(k)
    assert not bad, f"{len(bad)} non-exempt feature points differ, e.g. {sorted(bad)[:5]}"
    common = set(g) & set(o)
    if common:
        err = max(abs(float(g[k]) - float(o[k])) for k in common)
        assert err <= tol_r, f"point response error {err} > {tol_r}"
    return len(g), len(o)


# ---------------------------------------------------------------- generic chains
U32 = 2.0 ** -24  # unit roundoff of FP32


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def generic_reference(oracle_lib, spec, volume):
    """Oracle output of a generic chain and a per-pixel bound on the error of
    any FP32 evaluation that rounds each stage's result once per operation in
    the stated order.

    The bound is propagated stage by stage from the oracle's exact
    intermediates X and the incoming bound E (the input is exact, E = 0):
      stencil, n taps, fused multiply-adds: E' = |w| * E + gamma_n |w| * (|X| + E)
      window sum of nx x ny values (rows, then the row sums):
                                           E' = box(E) + gamma_{nx+ny} box(|X| + E)
      affine fma(a, x, b):                 E' = |a| E + u (|a| (|X| + E) + |b|)
      abs, clamp (1-Lipschitz, exact):     E' = E
      square:                              E' = E (2|X| + E) + u (|X| + E)^2
      sqrt(|x|), correctly rounded:        E' = min(sqrt(E), E / sqrt|X|) + u sqrt(|X| + E)
    where * is correlation with replicate borders and gamma_n = n u / (1 - n u)
    (the standard bound for a recursive sum; Higham, Accuracy and Stability of
    Numerical Algorithms, Sec. 3.1).  Returns (X_final, E_final), [T][H][W]
    float64.
    """
    from scipy import ndimage

    X = np.asarray(volume, np.float64)
    E = np.zeros_like(X)
    for st in spec:
        Y = oracle_lib.gchain([st], X)
        A = np.abs(X) + E
        if st[0] == "stencil":
            aw = np.abs(np.asarray(st[3], np.float64))
            g = _gamma(aw.size)
            corr = lambda Z: np.stack([ndimage.correlate(z, aw, mode="nearest") for z in Z])
            E = corr(E) + g * corr(A)
        elif st[0] == "box":
            size = (2 * st[2] + 1, 2 * st[1] + 1)
            area = size[0] * size[1]
            g = _gamma(size[0] + size[1])
            box = lambda Z: np.stack([ndimage.uniform_filter(z, size=size, mode="nearest") * area for z in Z])
            E = box(E) + g * box(A)
        else:
            kind = st[1]
            if kind == "affine":
                a, b = abs(st[2]), abs(st[3])
                E = a * E + U32 * (a * A + b)
            elif kind == "square":
                E = E * (2.0 * np.abs(X) + E) + U32 * A * A
            elif kind == "sqrtabs":
                with np.errstate(divide="ignore", invalid="ignore"):
                    lip = np.where(np.abs(X) > 0, E / np.sqrt(np.abs(X)), np.inf)
                E = np.minimum(np.sqrt(E), lip) + U32 * np.sqrt(A)
            # abs and clamp leave E unchanged
        X = Y
    return X, E


def assert_within_bound(gpu, ref, bound, what=""):
    """|gpu - ref| <= bound (with 1% slack for evaluating the bound itself in
    FP64), everywhere; reports the worst ratio."""
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    lim = bound * 1.01 + 1e-30
    bad = err > lim
    assert not bad.any(), (f"{what}: {int(bad.sum())} pixels outside the FP32 error bound, worst "
                           f"err {err[bad].max():.3e} at bound {lim[bad][np.argmax(err[bad])]:.3e}")
    nz = bound > 0
    return float((err[nz] / bound[nz]).max()) if nz.any() else 0.0
