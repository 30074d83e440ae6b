"""Comparison rules between the GPU library and the FP64 oracle.

Floating-point stages: |gpu - oracle| <= 1e-4 on a 0-255 scale, i.e. 1e-4 of
the stage's full-scale value for uint8 input divided by 255:
  gauss 255, sobel 4*255, gradmag sqrt(2)*4*255, products (4*255)^2,
  box sums 25*(4*255)^2, harris / threshold (25*(4*255)^2)^2.

Integer outputs (gray, mask, frame difference) and feature points are compared
exactly, except at pixels whose decision FP32 rounding can flip.  Two sets of
such pixels are computed from the oracle's FP64 response R and window sums:

* literal: the stated rule -- the response lies within 1e-5 of the threshold,
  read relatively (|R - thr| <= 1e-5 thr; an absolute 1e-5 is below FP32
  resolution at 1e8) -- plus the pixels whose suppression decision compares
  against such a pixel (a 3x3 neighbour that survives the threshold);
* wide: FP32 evaluates R = Sxx*Syy - Sxy^2 - k (Sxx+Syy)^2 with an error
  proportional to the size of its terms, M = |Sxx*Syy| + Sxy^2 + k (Sxx+Syy)^2,
  not to R, so a pixel is exempt when R lies within eps = 1e-5 max(thr, M) of
  the threshold, or within eps of a neighbour's response that could beat it.

Every differing pixel must lie in the wide set, and every differing pixel and
point also in the literal set; both set sizes and the number of differences
are returned so the tests can assert them.  Point responses agree within
1e-5 M at the point (the same error model).
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


OFFS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)]


def _neighbour_index(idx, shape, dy, dx):
    """Flat indices of the (dy, dx) neighbours (replicate border) of flat pixel
    indices idx of a [T][H][W] array."""
    T, H, W = shape
    t, r = np.divmod(idx, H * W)
    y, x = np.divmod(r, W)
    y = np.clip(y + dy, 0, H - 1)
    x = np.clip(x + dx, 0, W - 1)
    return (t * H + y) * W + x


def decision_sets(R, M, thr=THR):
    """(wide, literal) boolean [T][H][W] arrays of the pixels whose suppression
    decision FP32 rounding may flip (see the module docstring).  Only pixels
    that can survive the threshold have neighbour clauses, so they are
    evaluated on those pixels alone."""
    R = np.asarray(R, np.float64)
    shape = R.shape
    Rf = R.ravel()
    eps = REL * np.maximum(thr, np.asarray(M, np.float64).ravel())
    near = np.abs(Rf - thr) <= eps
    wide = near.copy()
    live = np.nonzero(Rf >= thr - eps)[0]
    lit = np.abs(Rf - thr) <= REL * thr
    lit_ext = lit.copy()
    live_lit = np.nonzero(Rf >= thr * (1.0 - REL))[0]
    for dy, dx in OFFS:
        q = _neighbour_index(live, shape, dy, dx)
        rp, ep, rq, eq = Rf[live], eps[live], Rf[q], eps[q]
        hit = (near[q] & (rq >= rp - ep - eq)) | ((rq >= thr - eq) & (np.abs(rp - rq) <= ep + eq))
        wide[live[hit]] = True
        q2 = _neighbour_index(live_lit, shape, dy, dx)
        lit_ext[live_lit[lit[q2]]] = True
    return wide.reshape(shape), lit_ext.reshape(shape)


def decision_exempt(R, M, thr=THR):
    """The wide set alone (boolean [T][H][W])."""
    return decision_sets(R, M, thr)[0]


def diff_exempt(mask_exempt):
    """Frame-difference pixels that depend on an exempt mask pixel (t or t-1)."""
    ex = mask_exempt.copy()
    ex[1:] |= mask_exempt[:-1]
    return ex


def point_key(pts):
    return {(int(p[0]), int(p[1]), int(p[2])) for p in pts}


def compare_points(gpu, ora, wide, literal, M):
    """Point sets equal outside exempt pixels (wide and literal sets); the
    responses of common points within 1e-5 M of the oracle's.  Returns a dict
    of counts and the worst response error as a fraction of its bound."""
    g = {k: r for k, r in zip(map(tuple, gpu[:, :3].astype(np.int64).tolist()), gpu[:, 3])}
    o = {k: r for k, r in zip(map(tuple, ora[:, :3].astype(np.int64).tolist()), ora[:, 3])}
    differ = sorted(set(g) ^ set(o))
    bad = [k for k in differ if not wide[k]]
    assert not bad, f"{len(bad)} feature points differ outside the FP32 exemption, e.g. {bad[:5]}"
    bad = [k for k in differ if not literal[k]]
    assert not bad, (f"{len(bad)} feature points differ whose response is not within 1e-5 of the threshold: " +
                     ", ".join(f"{k} R={o.get(k, g.get(k)):.9g}" for k in bad[:20]))
    common = sorted(set(g) & set(o))
    worst = 0.0
    if common:
        idx = tuple(np.array(common).T)
        rg = np.array([g[k] for k in common], np.float64)
        ro = np.array([o[k] for k in common], np.float64)
        lim = REL * np.maximum(np.asarray(M)[idx], THR)
        ratio = np.abs(rg - ro) / lim
        j = int(np.argmax(ratio))
        assert ratio[j] <= 1.0, (f"point {common[j]}: response {rg[j]:.9g} vs oracle {ro[j]:.9g}, "
                                 f"error {abs(rg[j] - ro[j]):.3g} > 1e-5 M = {lim[j]:.3g}")
        worst = float(ratio[j])
    return {"points_gpu": len(g), "points_oracle": len(o), "points_differ": len(differ),
            "response_err_over_bound": worst}


def compare_decisions(g, o, wide, literal, what="output"):
    """Integer decision outputs g (GPU) and o (oracle): every differing pixel is
    in the wide set and in the literal set.  Returns the number of differing
    pixels."""
    differ = g != o
    bad = differ & ~wide
    assert not bad.any(), f"{what}: {int(bad.sum())} pixels differ outside the FP32 exemption"
    bad = differ & ~literal
    if bad.any():
        locs = np.argwhere(bad)[:20].tolist()
        raise AssertionError(f"{what}: {int(bad.sum())} pixels differ outside the 1e-5-of-threshold rule: {locs}")
    return int(differ.sum())


def check_chain(oracle_lib, ops, vol, g, gp, skip=0):
    """GPU results of a chain ending in nms3 or framediff against the oracle.

    vol: the chain's input frames (any frame range of a video); g: the GPU's
    final output for the same frames ([T][H][W] uint8); gp: the GPU's points in
    those frames, t relative to the range's first frame.  The first `skip`
    frames are temporal halo (the oracle starts its frame difference there
    with m[-1] := m[0]) and are not compared.  Returns the counts: wide and
    literal exemption sets, differing pixels, points and the worst response
    error over its bound."""
    o, op_ = oracle_lib.chain(ops, vol)
    h = ops.index("harris")
    sums, _ = oracle_lib.chain(ops[:h], vol)
    R, _ = oracle_lib.chain(ops[:h + 1], vol)
    M = term_size(sums)
    del sums
    wide, lit = decision_sets(R[0], M)
    wf, lf = (diff_exempt(wide), diff_exempt(lit)) if ops[-1] == "framediff" else (wide, lit)
    n = compare_decisions(np.asarray(g)[skip:], o[0].astype(np.uint8)[skip:], wf[skip:], lf[skip:],
                          ops[-1] + " output")
    st = compare_points(gp[gp[:, 0] >= skip], op_[op_[:, 0] >= skip], wide, lit, M)
    st.update(n_wide=int(wide[skip:].sum()), n_literal=int(lit[skip:].sum()), px_differ=n)
    return st


def add_stats(total, st):
    for k, v in st.items():
        total[k] = max(total.get(k, 0.0), v) if k == "response_err_over_bound" else total.get(k, 0) + v
    return total


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
        if st[0] == "iir":
            E = iir_bound(st[1], X, Y, E)
        elif st[0] == "stencil":
            aw = np.abs(np.asarray(st[3], np.float64))
            g = _gamma(aw.size)
            if aw.ndim == 3:  # frame window: w[tau] on frame t - tau, the first frame replicated
                def corr(Z):
                    out = np.zeros_like(Z)
                    for tau in range(aw.shape[0]):
                        src = Z[np.maximum(np.arange(Z.shape[0]) - tau, 0)]
                        out += np.stack([ndimage.correlate(z, aw[tau], mode="nearest") for z in src])
                    return out
            else:
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


def iir_bound(a, X, Y, E):
    """Error bound of the IIR as the library evaluates it: the state in double
    precision, y = fma(a, x, (1 - a) y_prev) on the f32 inputs x (bound E),
    y[-1] := x[0], each output rounded once to f32:
      G[t] = |a| E[t] + (1 - a) G[t-1]
             + 2 u64 (|a| (|X[t]| + E[t]) + (1 - a) (|Y[t-1]| + G[t-1])),   G[-1] = E[0]
      F[t] = G[t] + u32 (|Y[t]| + G[t])
    from the exact input X and output Y ([T][H][W]); F bounds the f32 output."""
    a = float(a)
    b = 1.0 - a
    u64 = 2.0 ** -53
    F = np.zeros_like(E)
    yprev, gprev = np.abs(X[0]), E[0].copy()
    for t in range(X.shape[0]):
        G = (abs(a) * E[t] + b * gprev + 2 * u64 * (abs(a) * (np.abs(X[t]) + E[t]) + b * (yprev + gprev)))
        F[t] = G + U32 * (np.abs(Y[t]) + G)
        yprev, gprev = np.abs(Y[t]), G
    return F


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


def generic_full_scale(spec, s=255.0):
    """Largest output magnitude a generic chain can reach from inputs in
    [-s, s] (uint8 input: s = 255), stage by stage: a stencil scales it by
    sum |w|, a window sum by its area, affine by |a| (plus |b|), square
    squares it, sqrt-abs takes its root, abs keeps it, clamp maps [-s, s]
    into [clamp(-s), clamp(s)]."""
    for st in spec:
        if st[0] == "iir":
            continue  # a convex combination of earlier inputs: the range is kept
        if st[0] == "stencil":
            s *= float(np.abs(np.asarray(st[3], np.float64)).sum())
        elif st[0] == "box":
            s *= (2 * st[1] + 1) * (2 * st[2] + 1)
        elif st[1] == "affine":
            s = abs(st[2]) * s + abs(st[3])
        elif st[1] == "square":
            s = s * s
        elif st[1] == "sqrtabs":
            s = np.sqrt(s)
        elif st[1] == "clamp":
            c = lambda v: min(max(v, st[2]), st[3])
            s = max(abs(c(-s)), abs(c(s)))
    return float(s)


def north_star_tol(spec):
    """|gpu - oracle| allowed for a generic chain: 1e-4 on a 0-255 scale, i.e.
    1e-4 of the chain's full-scale output magnitude for uint8 input over 255."""
    return 1e-4 * generic_full_scale(spec) / 255.0
