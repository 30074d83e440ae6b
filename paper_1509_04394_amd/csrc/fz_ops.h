// Operation registry and fused-group geometry, shared by the host planner and
// the device kernels so that the on-chip footprint the planner prices is the
// one the launcher allocates.
#pragma once

#include <stdint.h>

#include "../../include/fz.h"

#if defined(__HIPCC__)
#define FZ_HD __host__ __device__
#else
#define FZ_HD
#endif

namespace fz {

// Access pattern of one operation (Sec. IV, Table I): window radius r (the
// output reads (2r+1) x (2r+1) input pixels), frames back rt, channel counts
// and element types in and out, and the Sec. V-A dependence on the predecessor.
struct OpInfo {
    int op, r, rt, in_ch, out_ch, in_dt, out_dt, dep;
    int ops_per_px;  // algorithmic arithmetic per output pixel (separable, no recompute)
};

FZ_HD constexpr OpInfo op_info(int op)
{
    switch (op) {
    case FZ_OP_RGB2GRAY: return {op, 0, 0, 3, 1, FZ_U8, FZ_U8, FZ_DEP_TT, 9};
    case FZ_OP_GAUSS5: return {op, 2, 0, 1, 1, FZ_U8, FZ_F32, FZ_DEP_TMT, 11};
    case FZ_OP_SOBEL3: return {op, 1, 0, 1, 2, FZ_F32, FZ_F32, FZ_DEP_TMT, 10};
    case FZ_OP_GRADMAG: return {op, 0, 0, 2, 1, FZ_F32, FZ_F32, FZ_DEP_TT, 3};
    case FZ_OP_PRODUCTS: return {op, 0, 0, 2, 3, FZ_F32, FZ_F32, FZ_DEP_TT, 3};
    case FZ_OP_BOXSUM5: return {op, 2, 0, 3, 3, FZ_F32, FZ_F32, FZ_DEP_TMT, 24};
    case FZ_OP_HARRIS: return {op, 0, 0, 3, 1, FZ_F32, FZ_F32, FZ_DEP_TT, 5};
    case FZ_OP_THRESHOLD: return {op, 0, 0, 1, 1, FZ_F32, FZ_F32, FZ_DEP_TT, 2};
    case FZ_OP_NMS3: return {op, 1, 0, 1, 1, FZ_F32, FZ_U8, FZ_DEP_TMT, 7};
    case FZ_OP_FRAMEDIFF: return {op, 0, 1, 1, 1, FZ_U8, FZ_U8, FZ_DEP_TT, 2};
    // generic stages: defaults only (radii, weights and kinds come with the stage)
    case FZ_OP_STENCIL: return {op, 1, 0, 1, 1, FZ_F32, FZ_F32, FZ_DEP_TMT, 9};
    case FZ_OP_BOX: return {op, 1, 0, 1, 1, FZ_F32, FZ_F32, FZ_DEP_TMT, 9};
    case FZ_OP_POINT: return {op, 0, 0, 1, 1, FZ_F32, FZ_F32, FZ_DEP_TT, 1};
    // IIR filter (Table II): a point operation over every earlier frame (rt = -1)
    case FZ_OP_IIR: return {op, 0, -1, 1, 1, FZ_F32, FZ_F32, FZ_DEP_TT, 2};
    default: return {0, 0, 0, 0, 0, 0, 0, 0, 0};
    }
}

FZ_HD constexpr int dt_bytes(int dt) { return dt == FZ_F32 ? 4 : 1; }
FZ_HD constexpr bool is_generic_op(int op)
{
    return op == FZ_OP_STENCIL || op == FZ_OP_BOX || op == FZ_OP_POINT || op == FZ_OP_IIR;
}

// The stage sequences the kernels are compiled for.  A user chain is any
// contiguous part of one of them.
enum { CHAIN_HARRIS = 0, CHAIN_GRAD = 1, N_CHAINS = 2 };

FZ_HD constexpr int chain_len(int ch) { return ch == CHAIN_HARRIS ? 9 : 3; }

FZ_HD constexpr int chain_op(int ch, int i)
{
    if (ch == CHAIN_HARRIS) {
        switch (i) {
        case 0: return FZ_OP_RGB2GRAY;
        case 1: return FZ_OP_GAUSS5;
        case 2: return FZ_OP_SOBEL3;
        case 3: return FZ_OP_PRODUCTS;
        case 4: return FZ_OP_BOXSUM5;
        case 5: return FZ_OP_HARRIS;
        case 6: return FZ_OP_THRESHOLD;
        case 7: return FZ_OP_NMS3;
        case 8: return FZ_OP_FRAMEDIFF;
        default: return 0;
        }
    }
    switch (i) {
    case 0: return FZ_OP_GAUSS5;
    case 1: return FZ_OP_SOBEL3;
    case 2: return FZ_OP_GRADMAG;
    default: return 0;
    }
}

// Halo still needed after stage s of group [A..B]: the sum of the radii of the
// later window stages.  Window radii add when stencils are composed (a 5x5
// smoothing followed by a 3x3 gradient reads 7x7 input pixels), so the input
// box of the group grows by the sum of the radii per side (Sec. VI-C gives the
// per-kernel growth; the group's growth is their sum).
FZ_HD constexpr int halo_after(int ch, int s, int B)
{
    int h = 0;
    for (int j = s + 1; j <= B; ++j) h += op_info(chain_op(ch, j)).r;
    return h;
}
FZ_HD constexpr int group_halo(int ch, int A, int B) { return halo_after(ch, A - 1, B); }
FZ_HD constexpr int group_halo_t(int ch, int A, int B)
{
    int h = 0;
    for (int j = A; j <= B; ++j) h += op_info(chain_op(ch, j)).rt;
    return h;
}
FZ_HD constexpr bool group_has_window(int ch, int A, int B)
{
    for (int j = A; j <= B; ++j)
        if (op_info(chain_op(ch, j)).r > 0) return true;
    return false;
}
FZ_HD constexpr bool is_window(int ch, int s) { return op_info(chain_op(ch, s)).r > 0; }

// Channels held per pixel in the on-chip buffer right after window stage s and
// the point ops that follow it inside the group (they run in registers).
FZ_HD constexpr int channels_after_step(int ch, int s, int B)
{
    int c = op_info(chain_op(ch, s)).out_ch;
    for (int j = s + 1; j <= B && !is_window(ch, j); ++j) c = op_info(chain_op(ch, j)).out_ch;
    return c;
}
// Channels of the loaded input after the leading point ops of the group.
FZ_HD constexpr int channels_after_load(int ch, int A, int B)
{
    int c = op_info(chain_op(ch, A)).in_ch;
    for (int j = A; j <= B && !is_window(ch, j); ++j) c = op_info(chain_op(ch, j)).out_ch;
    return c;
}

// On-chip footprint (floats) of the LDS tile engine for group [A..B] with an
// output tile TW x TH: two buffers, each large enough for the largest
// (cells x channels) of any step (a load, a horizontal pass, a window output).
FZ_HD constexpr int engine_buffer_floats(int ch, int A, int B, int TW, int TH)
{
    int H = group_halo(ch, A, B);
    int mx = (TW + 2 * H) * (TH + 2 * H) * channels_after_load(ch, A, B);
    for (int s = A; s <= B; ++s) {
        if (!is_window(ch, s)) continue;
        int hin = halo_after(ch, s - 1, B), hout = halo_after(ch, s, B);
        int cin = op_info(chain_op(ch, s)).in_ch;
        // horizontal-pass intermediate: input rows x output columns
        int tmp = (TH + 2 * hin) * (TW + 2 * hout) * cin;
        int outc = (TW + 2 * hout) * (TH + 2 * hout) * channels_after_step(ch, s, B);
        if (hout == 0) outc = 0;  // the last window step writes global memory
        if (tmp > mx) mx = tmp;
        if (outc > mx) mx = outc;
    }
    return mx;
}
FZ_HD constexpr int engine_lds_bytes(int ch, int A, int B, int TW, int TH)
{
    return group_has_window(ch, A, B) ? 2 * 4 * engine_buffer_floats(ch, A, B, TW, TH) : 0;
}

// Tile shapes the LDS engine is compiled for (output box x by y).
constexpr int N_TILES = 3;
FZ_HD constexpr int tile_w(int t) { return t == 0 ? 64 : (t == 1 ? 32 : 64); }
FZ_HD constexpr int tile_h(int t) { return t == 0 ? 16 : (t == 1 ? 32 : 32); }

constexpr int BLOCK_THREADS = 256;

}  // namespace fz
