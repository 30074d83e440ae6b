// Generic single-channel chains: point, weighted-stencil and window-sum stages
// whose radii, weights and point kinds are given at plan time (the Table I
// access classes with free parameters).  Shared by the planner, which prices
// a group with the on-chip footprint below, and by the launcher.
#pragma once

#include <stdint.h>

#include "fz_ops.h"

namespace fz {

constexpr int G_MAX_STAGES = 16;
constexpr int G_MAX_R = 3;
constexpr int G_MAX_WEIGHTS = G_MAX_STAGES * (2 * G_MAX_R + 1) * (2 * G_MAX_R + 1);

enum { G_POINT = 0, G_STENCIL = 1, G_BOX = 2 };

struct GStage {
    int32_t kind;    // G_POINT / G_STENCIL / G_BOX
    int32_t rx, ry;  // window radii (0 for point stages)
    int32_t pk;      // FZ_POINT_* kind of a point stage
    float a, b;      // point-stage parameters
    int32_t woff;    // first weight of a stencil stage in GParams::w
    int32_t pad;
};

// Kernel arguments of one generic group: the stage list and every stencil
// weight travel by value (at most 16 stages of radius <= 3: 784 weights,
// under 4 KB in all), so a run needs no device buffer for them.
struct GParams {
    const void* in;
    float* out;
    int32_t W, H, T, in_u8;
    int32_t n;         // stages in the group
    int32_t hx, hy;    // group halo: the sums of the window radii
    int32_t tiles_x, tiles_y, pad;
    GStage st[G_MAX_STAGES];
    float w[G_MAX_WEIGHTS];
};

// LDS of the generic tile kernel: the input box (TW + 2hx) x (TH + 2hy) as
// f32, doubled when a window step has to hand its output to a later window
// step (the last window step writes global memory directly), plus GEN_PAD
// floats: a thread computes five neighbouring cells of a row and may read the
// row up to four cells past the last one it needs.
constexpr int GEN_PAD = 4;
FZ_HD constexpr int generic_lds_bytes(int tw, int th, int hx, int hy, int nwin)
{
    return nwin == 0 ? 0 : ((nwin >= 2 ? 2 : 1) * (tw + 2 * hx) * (th + 2 * hy) + GEN_PAD) * 4;
}

// Algorithmic arithmetic per output pixel of a generic stage: one
// multiply-add per stencil tap, one add per window-sum element, one operation
// per point stage (two for a clamp).
FZ_HD constexpr int generic_ops(int kind, int rx, int ry, int pk)
{
    return kind == G_POINT ? (pk == FZ_POINT_CLAMP ? 2 : 1) : (2 * rx + 1) * (2 * ry + 1);
}

}  // namespace fz
