// Work layout of the generated kernels: cells per thread of each window
// stage and the LDS row pitch that keeps the stages' LDS accesses off shared
// banks.  Host code; the generator (jit.cpp) and the planner's LDS sizing use
// it.
#include <algorithm>
#include <vector>

#include "jit_layout.h"

namespace fz {

// Rows of outputs per thread of a window stage: each thread computes a block
// of GQ x gr cells (gr <= 2), so the input rows it reads and (for a window
// sum) the row sums it forms serve gr output rows.  Chosen by a count of wave
// instructions: wave passes (ceil(items / 64)) times an estimate of the
// instructions per item.
static int pick_rows(const GStage& s, int ow, int oh, int trail_ops, bool last, int GQ)
{
    const int nq = (ow + GQ - 1) / GQ;
    int best = 1;
    long best_cost = -1;
    for (int gr = 1; gr <= 2 && gr <= oh; ++gr) {  // four rows: ~30 more registers, a wave fewer per SIMD
        const int items = nq * ((oh + gr - 1) / gr);
        const int rows_in = gr + 2 * s.ry;
        long per = 14 + (long)GQ * gr * (1 + trail_ops + (last ? 1 : 0));
        if (s.kind == G_STENCIL)
            per += (long)GQ * gr * (2 * s.rx + 1) * (2 * s.ry + 1) * (s.rt + 1);
        else
            per += (long)(s.rt + 1) * (rows_in * GQ * 2 * s.rx + (long)gr * GQ * 2 * s.ry);
        if (last) per += 4L * gr;
        const long cost = (long)((items + 63) / 64) * per;
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = gr;
        }
    }
    return best;
}

std::vector<WinStep> win_steps(const GStage* st, int n, int TW, int TH, int HX, int HY)
{
    std::vector<WinStep> w;
    int i = 0, hx = HX, hy = HY;
    while (i < n && !g_is_window(st[i].kind)) ++i;
    while (i < n) {
        int j = i + 1, trail_ops = 0;
        while (j < n && !g_is_window(st[j].kind)) trail_ops += st[j++].kind == G_IIR ? 8 : 2;
        WinStep s;
        s.i = i;
        s.j = j;
        s.last = j == n;
        s.ohx = hx - st[i].rx;
        s.ohy = hy - st[i].ry;
        // cells across per thread: five (fewer LDS reads per output), four in
        // the last stage, whose rows then go out as aligned 16-byte stores
        s.gq = s.last ? 4 : 5;
        s.gr = pick_rows(st[i], TW + 2 * s.ohx, TH + 2 * s.ohy, trail_ops, s.last, s.gq);
        w.push_back(s);
        hx = s.ohx;
        hy = s.ohy;
        i = j;
    }
    return w;
}

// LDS row pitch of a group's buffers (cells per box row, at least the box
// width rounded up to whole four-cell groups).  A window stage's thread reads and writes its cell block at
// (row, column) = (BY + cy, BX + cx) plus offsets common to every lane, so
// the bank conflicts of each of its LDS instructions are those of the lanes'
// cy * pitch + cx over 32 banks of 4 bytes, per 32 lanes; the pitch with the
// fewest conflict cycles, weighted by each stage's reads and writes per
// item, is taken among the next 32.  (On the 800x600x64 generic chain the
// pitch 83 for a 68-cell box cut the LDS bank-conflict cycles from 62% to 36%
// of the LDS-active cycles and the kernel from 68 to 59 us; restricting the
// pitch to multiples of 4, for aligned 16-byte stores of the input box, gave
// 72 and 71 us.)
int jit_pitch(const GStage* st, int n, int TW, int TH, int HX, int HY)
{
    // at least the four-cell groups' width (leading IIR states are indexed by group)
    const int RW = TW + 2 * HX, S = (4 - HX % 4) % 4, lp0 = std::max(RW, (RW + S + 3) / 4 * 4);
    const std::vector<WinStep> w = win_steps(st, n, TW, TH, HX, HY);
    int best = lp0;
    long best_cost = -1;
    for (int lp = lp0; lp < lp0 + 32; ++lp) {
        long cost = 0;
        for (const WinStep& s : w) {
            const GStage& g = st[s.i];
            const int OW = TW + 2 * s.ohx, OH = TH + 2 * s.ohy;
            const int NQ = (OW + s.gq - 1) / s.gq, NR = (OH + s.gr - 1) / s.gr, items = NQ * NR;
            const long per_item = (long)(g.rt + 1) * (s.gr + 2 * g.ry) * (s.gq + 2 * g.rx) + (s.last ? 0 : s.gr * s.gq);
            long cycles = 0;
            for (int h0 = 0; h0 < items; h0 += 32) {
                // the lanes' addresses are distinct (distinct cells of the stage's output region)
                int count[32] = {0}, deg = 1;
                for (int e = h0; e < items && e < h0 + 32; ++e) {
                    const int ry = e / NQ, cx = (e - ry * NQ) * s.gq, cy = std::min(ry * s.gr, OH - s.gr);
                    deg = std::max(deg, ++count[(cy * lp + cx) & 31]);
                }
                cycles += deg;
            }
            cost += cycles * per_item;
        }
        // a wider pitch also costs LDS: count its share of a conflict-free cycle per cell
        cost = cost * 64 + (long)(lp - lp0);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = lp;
        }
    }
    return best;
}

// LDS layout of a generated kernel: march_layout's, except that the IIRs
// before the first window stage keep their states in registers and take no
// LDS (their buf is -1).  Returns the floats used (the caller adds GEN_PAD).
int jit_layout(GStage* st, int n, int cells)
{
    int off = 0, shared[2] = {-1, -1}, alt = 0;
    bool seen_window = false;
    for (int j = 0; j < n; ++j) {
        GStage& s = st[j];
        s.buf = -1;
        s.slots = 0;
        if (g_is_window(s.kind)) {
            seen_window = true;
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
        } else if (s.kind == G_IIR && seen_window) {
            off += off & 1;  // 8-byte alignment of the double state
            s.buf = off;
            off += 2 * cells;
        }
    }
    return off;
}

}  // namespace fz
