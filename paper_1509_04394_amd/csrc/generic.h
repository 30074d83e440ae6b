// Generic single-channel chains: point, weighted-stencil, window-sum and IIR
// stages whose radii, weights and parameters are given at plan time (the
// Table I access classes with free parameters, and Table II's IIR filter).
// Shared by the planner, which prices a group with the on-chip footprint
// below, and by the launcher.
#pragma once

#include <stdint.h>

#include "fz_ops.h"

namespace fz {

constexpr int G_MAX_STAGES = 16;
constexpr int G_MAX_R = 3;
constexpr int G_MAX_RT = 3;  // frames back of a spatio-temporal stencil
constexpr int G_MAX_WEIGHTS = G_MAX_STAGES * (2 * G_MAX_R + 1) * (2 * G_MAX_R + 1);

enum { G_POINT = 0, G_STENCIL = 1, G_BOX = 2, G_IIR = 3 };

FZ_HD constexpr bool g_is_window(int kind) { return kind == G_STENCIL || kind == G_BOX; }
FZ_HD constexpr int g_kind(int op)
{
    return op == FZ_OP_POINT ? G_POINT : (op == FZ_OP_STENCIL ? G_STENCIL : (op == FZ_OP_BOX ? G_BOX : G_IIR));
}

struct GStage {
    int32_t kind;        // G_POINT / G_STENCIL / G_BOX / G_IIR
    int32_t rx, ry, rt;  // window radii; frames back of a stencil (0 = this frame only)
    int32_t pk;          // FZ_POINT_* kind of a point stage
    float a, b;          // point-stage parameters; IIR: a
    int32_t woff;        // first weight of a stencil stage in GParams::w
    int32_t buf;         // LDS offset (floats) of a window stage's input ring or an IIR's (double) state
    int32_t slots;       // marching kernel: frames the input ring of a window stage holds (rt + 1)
    int32_t pad[2];
};

// Kernel arguments of one generic group: the stage list and every stencil
// weight travel by value (at most 784 weights per group, under 4 KB of
// arguments in all), so a run needs no device buffer for them.
struct GParams {
    const void* in;
    float* out;
    int32_t W, H, T, in_u8;
    int32_t n;          // stages in the group
    int32_t hx, hy;     // group halo: the sums of the window radii
    int32_t tiles_x, tiles_y;
    int32_t tt;         // marching kernel: output frames per work item
    int32_t ht;         // marching kernel: temporal halo, the sum of the stencils' frames back
    int32_t ck_n;       // IIR stages restored from checkpoints (0: none)
    const double* ckpt; // IIR checkpoints: [chunk - 1][IIR][H][W] states after frame chunk * tt - 1
    GStage st[G_MAX_STAGES];
    float w[G_MAX_WEIGHTS];
};
static_assert(sizeof(GParams) <= 4096, "generic kernel arguments must stay within 4 KB");

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

// LDS layout of the frame-marching kernel (groups with a temporal stage) over
// a box of `cells` floats: every window stage reads its input from LDS; the
// inputs of stages that look only at the current frame alternate between two
// shared buffers, a stencil that looks rt frames back keeps a ring of its last
// rt + 1 input frames of its own, and every IIR stage keeps its running state
// (one double per box cell, two floats, at an even offset).  Fills
// GStage::buf / slots and returns the floats used (the caller adds GEN_PAD).
FZ_HD inline int march_layout(GStage* st, int n, int cells)
{
    int off = 0, shared[2] = {-1, -1}, alt = 0;
    for (int j = 0; j < n; ++j) {
        GStage& s = st[j];
        s.buf = -1;
        s.slots = 0;
        if (g_is_window(s.kind)) {
            s.slots = s.rt + 1;
            if (s.rt == 0) {
                if (shared[alt] < 0) {
                    shared[alt] = off;
                    off += cells;
                }
                s.buf = shared[alt];
                alt ^= 1;
            } else {
                s.buf = off;
                off += s.slots * cells;
            }
        } else if (s.kind == G_IIR) {
            off += off & 1;  // 8-byte alignment of the double state
            s.buf = off;
            off += 2 * cells;
        }
    }
    return off;
}

// Algorithmic arithmetic per output pixel of a generic stage: one
// multiply-add per stencil tap (over every frame it reads), one add per
// window-sum element, one operation per point stage (two for a clamp), two
// for an IIR step (a multiply and a multiply-add).
FZ_HD constexpr int generic_ops(int kind, int rx, int ry, int pk, int rt = 0)
{
    return kind == G_POINT ? (pk == FZ_POINT_CLAMP ? 2 : 1)
                           : (kind == G_IIR ? 2 : (2 * rx + 1) * (2 * ry + 1) * (rt + 1));
}

// Stage descriptors of stages a..b of a generic chain (weights not copied;
// woff, buf and slots left 0).  IIR: a = param[0] (the kernels form 1 - a in
// double precision, exactly).  Returns the weights the group's stencils hold
// (over every frame they read).
inline int g_stage_list(const fz_stage* st, int a, int b, GStage* out)
{
    int nw = 0;
    for (int j = a; j <= b; ++j) {
        const fz_stage& f = st[j];
        GStage d{};
        d.kind = g_kind(f.op);
        d.rx = f.rx;
        d.ry = f.ry;
        d.rt = (d.kind == G_STENCIL && f.rt > 0) ? f.rt : 0;
        if (d.kind == G_IIR) {
            d.a = f.param[0];
        } else {
            d.pk = (int)f.param[0];
            d.a = f.param[1];
            d.b = f.param[2];
        }
        if (d.kind == G_STENCIL) nw += (2 * f.rx + 1) * (2 * f.ry + 1) * (d.rt + 1);
        out[j - a] = d;
    }
    return nw;
}
// A group with an IIR or a stencil that looks back marches through frames.
inline bool g_temporal(const GStage* st, int n, bool* has_iir = nullptr, int* ht = nullptr)
{
    bool iir = false;
    int back = 0;
    for (int j = 0; j < n; ++j) {
        iir |= st[j].kind == G_IIR;
        back += st[j].rt;
    }
    if (has_iir) *has_iir = iir;
    if (ht) *ht = back;
    return iir || back > 0;
}

// Output tiles of the generated (hipRTC) kernels, x by y.
constexpr int N_JIT_TILES = 5;
// Work items a generated kernel without temporal stages keeps when it takes
// several frames per item (two rounds of four 256-thread workgroups per CU).
constexpr int JIT_FILL_ITEMS = 2048;
extern const int JIT_TILES[N_JIT_TILES][2];
// LDS row pitch (cells) of a generated kernel's buffers for stages st[0..n)
// on TW x TH tiles with halos HX, HY (at least TW + 2 HX rounded up to the
// box's four-cell groups, so a row of IIR states by group fits).
int jit_pitch(const GStage* st, int n, int TW, int TH, int HX, int HY);
// A generated kernel's LDS layout (march_layout's, with the IIRs before the
// first window stage in registers instead): sets buf / slots, returns floats.
int jit_layout(GStage* st, int n, int cells);

// A group whose IIR stages all come before its first window stage, and whose
// stencils do not look back, can run in frame runs shorter than the clip: a
// first pass marches the IIRs alone over every pixel and writes their state at
// the end of every run (a checkpoint), and each work item of the group starts
// its run from the checkpoint of the run before.  Returns the number of such
// IIR stages, 0 if the group does not qualify.
inline int g_ckpt_iirs(const GStage* st, int n)
{
    int lead = 0;
    bool window = false;
    for (int j = 0; j < n; ++j) {
        if (st[j].rt > 0) return 0;
        if (g_is_window(st[j].kind)) window = true;
        if (st[j].kind == G_IIR) {
            if (window) return 0;
            ++lead;
        }
    }
    return window ? lead : 0;
}

// Work items that fill the device: 256 CUs x 4 SIMDs, one 256-thread
// workgroup (four wavefronts) per SIMD slot.
constexpr int G_FILL_ITEMS = 1024;

}  // namespace fz
