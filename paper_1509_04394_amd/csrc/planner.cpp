// Host planner and C-ABI entry points that do not touch the device.
//
// Sec. VI-A: kernels with only thread-to-thread or thread-to-multi-thread
// dependences form fusable sets; within a set every contiguous group of
// kernels is a candidate fused kernel (n(n+1)/2 of them, Fig. 5) and the
// partition of least total cost is chosen.  Because the candidates are the
// contiguous runs of a sequence, an exact cover by chosen candidates is a path
// through the cut positions 0..n, and the minimum is a shortest path solved by
// dynamic programming over the last cut, with no integer-programming solver.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "fz_internal.h"
#include "generic.h"
#include "rowgeom.h"

namespace fz {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

fz_status fail(fz_status code, const std::string& msg)
{
    g_err = msg;
    return code;
}

static const double kInf = std::numeric_limits<double>::infinity();

static int op_bytes_in(int op)
{
    const OpInfo o = op_info(op);
    return o.in_ch * dt_bytes(o.in_dt);
}
static int op_bytes_out(int op)
{
    const OpInfo o = op_info(op);
    return o.out_ch * dt_bytes(o.out_dt);
}

// Data utilisation of an output box x*y*t with growth 2H per axis and Ht
// frames (Eq. 3).
static double data_utilisation(int x, int y, int t, int H, int Ht)
{
    return (double)x * y * t / ((double)(x + 2 * H) * (y + 2 * H) * (t + Ht));
}

Segment price_group(const fz_plan& p, int a, int b, int req_w, int req_h, int req_tpb, int req_engine)
{
    Segment s{};
    s.first = a;
    s.last = b;
    s.cfirst = p.offset + a;
    s.clast = p.offset + b;
    s.cost = kInf;
    s.tile = -1;
    for (int j = a + 1; j <= b; ++j)
        if (p.stages[j].dep == FZ_DEP_KK) return s;  // kernel-to-kernel: never fused (Sec. VI-A)
    if (p.generic) return price_generic(p, a, b, req_w, req_h, req_tpb, req_engine);
    const int ch = p.chain, A = s.cfirst, B = s.clast;
    s.halo = s.halo_y = group_halo(ch, A, B);
    s.halo_t = group_halo_t(ch, A, B);
    s.streaming = group_has_window(ch, A, B) ? 0 : 1;
    s.tpb = req_tpb > 0 ? req_tpb : (s.halo_t > 0 ? 8 : 1);
    if (s.tpb > p.T) s.tpb = p.T;
    // row-marching: the Harris-chain kernel for its groups, the generic kernel
    // (two columns per lane) for every other group with a window stage
    const bool rgb_in = chain_op(ch, A) == FZ_OP_RGB2GRAY;
    const bool row_special = row_group(ch, A, B) && row_strips_best(p.W, rgb_in) > 0;
    const bool row_generic = !row_special && rowgen_group(ch, A, B) && row_strips(p.W, 2, s.halo) > 0;
    const bool row_ok = !s.streaming && (row_special || row_generic) && p.H >= 8 && req_engine != FZ_ENGINE_TILE &&
                        req_w == 0;
    if (s.streaming) {
        s.engine = FZ_ENGINE_STREAM;
        s.lds_bytes = 0;
        s.tile_w = s.tile_h = 0;
    } else if (row_ok) {
        s.engine = FZ_ENGINE_ROW;
        s.row_gen = row_generic ? 1 : 0;
        const bool diff = chain_op(ch, B) == FZ_OP_FRAMEDIFF;
        s.row_k = row_generic ? 2 : row_strips_best(p.W, rgb_in);
        s.nstrips = row_strips(p.W, s.row_k, row_generic ? s.halo : ROW_HX);
        const int slots = row_generic ? ROW_SLOTS_GENERIC : row_slots(s.row_k, rgb_in);
        const RowShape rs = row_shape(p.H, p.T, s.nstrips, diff, req_h, req_tpb, slots);
        if (rs.band_h == 0) {
            s.refused = 1;
            return s;
        }
        s.tpb = rs.tt;
        s.nchunks = (p.T + s.tpb - 1) / s.tpb;
        s.tile_h = rs.band_h;
        s.nbands = (p.H + s.tile_h - 1) / s.tile_h;
        s.tile_w = 64 * s.row_k;
        s.lds_bytes = diff ? row_lds_bytes(s.tile_h) : 0;
        if (s.lds_bytes > p.lds_budget) return s;
        s.tile = 0;
    } else {
        s.engine = FZ_ENGINE_TILE;
        double best_du = -1.0;
        for (int t = 0; t < N_TILES; ++t) {
            const int tw = tile_w(t), th = tile_h(t);
            if (req_w > 0 && (tw != req_w || th != req_h)) continue;
            const int lds = engine_lds_bytes(ch, A, B, tw, th);
            if (lds > p.lds_budget) continue;
            const double du = data_utilisation(tw, th, s.tpb, s.halo, s.halo_t);
            if (du > best_du) {
                best_du = du;
                s.tile = t;
                s.tile_w = tw;
                s.tile_h = th;
                s.lds_bytes = lds;
            }
        }
        if (s.tile < 0) return s;  // no compiled tile fits the on-chip budget
    }
    // Compulsory traffic (Eq. 2 per group): the group's input once, its output
    // once; a multi-frame group re-reads its temporal halo once per frame run.
    const double bin = op_bytes_in(p.stages[a].op), bout = op_bytes_out(p.stages[b].op);
    // (the Harris row kernel's frame-difference groups exchange the frame
    // before a run between items instead: no re-read)
    const bool exchange = s.engine == FZ_ENGINE_ROW && !s.row_gen && chain_op(ch, B) == FZ_OP_FRAMEDIFF;
    const double temporal =
        s.halo_t > 0 && !exchange ? bin * s.halo_t / (s.streaming ? 1.0 : (double)s.tpb) : 0.0;
    s.bytes_per_px = bin + bout + temporal;
    s.cost = s.bytes_per_px * (double)p.W * p.H * p.T;
    return s;
}

// Sec. VI-E, Eq. 6: among boxes x * x * t of fixed volume x^2 t = beta, the one
// whose input box (x + 2 dx)^2 (t + dt) is least (dx: halo per side, dt:
// frames of temporal halo; with the halo per side, Eq. 6 is exactly this
// minimiser).  Degenerate halos: no temporal halo -> the flattest box (t = 1);
// no spatial halo -> the thinnest (x = 1).
void eq6_box(double beta, double dx, double dt, double* x, double* t)
{
    if (dt <= 0.0) {
        *t = 1.0;
        *x = sqrt(beta);
    } else if (dx <= 0.0) {
        *x = 1.0;
        *t = beta;
    } else {
        *x = cbrt(2.0 * beta * dx / dt);
        *t = cbrt(beta) * pow(dt / dx, 2.0 / 3.0) / pow(2.0, 2.0 / 3.0);
    }
}

// A generic group: halos are the sums of its window radii per axis, its
// temporal halo the sum of its stencils' frames back.
//  * Point stages only: one streaming pass; with an IIR, one thread per run of
//    four pixels marches through every frame.
//  * A window stage and no temporal stage: the LDS tile kernel, the tile of
//    best data utilisation (Eq. 3) that fits the budget.
//  * A window stage and a temporal stage: the frame-marching tile kernel.  Its
//    on-chip footprint does not grow with the frame run (each stencil keeps
//    only its rt + 1 input frames), so the frame run is set by how many work
//    items fill the device instead: Eq. 6 with beta = W H T / G_FILL_ITEMS
//    output pixels per item gives t; then the tile of best Eq. 3 utilisation
//    for that t, discounted by the idle share of the device when the tile
//    leaves fewer work items than fill it.  IIRs that all come before the
//    first window stage (and no stencil looking back) are checkpointed: a
//    first pass writes their state at every run boundary and the runs are the
//    longest power of two (at least 8 frames) that leaves two fills of work
//    items.  Any other IIR makes the work items march the whole clip (t = T).
// Cost: compulsory bytes (input once, output once, the temporal halo re-read
// once per frame run), times G_FILL_ITEMS / items when a marching group has
// fewer work items than fill the device (its frames are a sequential chain
// per item, so the idle share of the device is lost time).  A group whose
// stencil weights exceed the kernel-argument store, or that asks for a frame
// run an IIR cannot keep, is not allowed.
Segment price_generic(const fz_plan& p, int a, int b, int req_w, int req_h, int req_tpb, int req_engine)
{
    Segment s{};
    s.first = s.cfirst = a;
    s.last = s.clast = b;
    s.cost = kInf;
    s.tile = -1;
    for (int j = a + 1; j <= b; ++j)
        if (p.stages[j].dep == FZ_DEP_KK) return s;
    GStage st[G_MAX_STAGES];
    const int n = b - a + 1;
    if (g_stage_list(p.stages.data(), a, b, st) > G_MAX_WEIGHTS) return s;
    int hx = 0, hy = 0, nwin = 0, ht = 0;
    bool iir = false;
    const bool temporal = g_temporal(st, n, &iir, &ht);
    for (int j = 0; j < n; ++j)
        if (g_is_window(st[j].kind)) {
            hx += st[j].rx;
            hy += st[j].ry;
            ++nwin;
        }
    s.halo = hx;
    s.halo_y = hy;
    s.halo_t = ht;
    s.tpb = 1;
    s.streaming = nwin == 0;
    const int n_ck = g_ckpt_iirs(st, n);  // leading IIRs that can resume from checkpoints
    if (iir && !n_ck && nwin > 0 && req_tpb > 0 && req_tpb < p.T) {
        s.refused = 2;  // an IIR after a window stage needs every earlier frame: whole-clip work items
        return s;
    }
    const double P = (double)p.W * p.H;
    double items = 0.0;
    if (s.streaming) {
        s.engine = FZ_ENGINE_STREAM;
        if (iir) {
            s.tpb = p.T;
            items = ceil(P / (4.0 * BLOCK_THREADS));
        }
    } else {
        // window groups: the compiled tiles of the tile kernels, or the generated kernels' tiles
        const bool jit = req_engine == FZ_ENGINE_JIT;
        s.engine = jit ? FZ_ENGINE_JIT : FZ_ENGINE_TILE;
        const int ntiles = jit ? N_JIT_TILES : N_TILES;
        int tt_fixed = 1;
        if (iir && !n_ck) {
            tt_fixed = p.T;
        } else if (temporal && !n_ck) {
            if (req_tpb > 0) {
                tt_fixed = std::min(req_tpb, p.T);
            } else {
                // Eq. 6 for a box of the work one item does when the items fill the device
                // once (four times for a generated kernel: on the 800x600x1000 look-back chain
                // its 16-frame runs took 2.41 ms against 2.51 at the single fill's 44)
                double x, t;
                eq6_box(P * p.T / (G_FILL_ITEMS * (jit ? 4.0 : 1.0)), 0.5 * (hx + hy), ht, &x, &t);
                tt_fixed = (int)std::min<double>(std::max(1.0, std::floor(t + 0.5)), p.T);
            }
        }
        double best_du = -1.0;
        int best_tt = tt_fixed;
        for (int t = 0; t < ntiles; ++t) {
            const int tw = jit ? JIT_TILES[t][0] : tile_w(t), th = jit ? JIT_TILES[t][1] : tile_h(t);
            if (req_w > 0 && (tw != req_w || th != req_h)) continue;
            const int cells = (tw + 2 * hx) * (th + 2 * hy);
            // a generated kernel: the marching layout (either kind of group) at its LDS row pitch
            const int lds = jit ? (jit_layout(st, n, jit_pitch(st, n, tw, th, hx, hy) * (th + 2 * hy)) + GEN_PAD) * 4
                            : temporal ? (march_layout(st, n, cells) + GEN_PAD) * 4
                                       : generic_lds_bytes(tw, th, hx, hy, nwin);
            if (lds > p.lds_budget) continue;
            const double tiles = ceil((double)p.W / tw) * ceil((double)p.H / th);
            int tt = tt_fixed;
            if (n_ck) {
                // checkpointed IIRs: the longest power-of-two run (at least 8 frames) that still
                // leaves two fills of work items (eight for a generated kernel: on the paper's
                // five-kernel chain at 800x600x1000 its 16-frame runs took 1.49 ms against 1.60 at
                // 64); each run boundary costs a checkpoint
                if (req_tpb > 0) {
                    tt = std::min(req_tpb, p.T);
                } else {
                    const double fills = jit ? 8.0 : 2.0;
                    tt = 8;
                    while (tt * 2 <= p.T && tiles * ceil((double)p.T / (tt * 2)) >= fills * G_FILL_ITEMS) tt *= 2;
                    tt = std::min(tt, p.T);
                }
            }
            double du = (double)tw * th / ((double)cells);
            if (temporal) {
                du *= (double)tt / (tt + (iir ? 0 : ht));
                // under-filled marching groups lose the idle share of the device
                const double it = tiles * ceil((double)p.T / tt);
                if (it < G_FILL_ITEMS) du *= it / G_FILL_ITEMS;
            }
            if (du > best_du) {
                best_du = du;
                best_tt = tt;
                s.tile = t;
                s.tile_w = tw;
                s.tile_h = th;
                s.lds_bytes = lds;
            }
        }
        if (s.tile < 0) return s;
        if (temporal) {
            s.tpb = best_tt;
            items = ceil((double)p.W / s.tile_w) * ceil((double)p.H / s.tile_h) * ceil((double)p.T / s.tpb);
            s.ckpt = n_ck > 0 && s.tpb < p.T;
        } else if (jit) {
            // a generated kernel marches a few frames per work item (its set-up
            // and the last frame's drain amortised): up to four, while at
            // least JIT_FILL_ITEMS work items remain
            const double tiles = ceil((double)p.W / s.tile_w) * ceil((double)p.H / s.tile_h);
            if (req_tpb > 0) {
                s.tpb = std::min(req_tpb, p.T);
            } else {
                s.tpb = 4;
                while (s.tpb > 1 && tiles * ceil((double)p.T / s.tpb) < JIT_FILL_ITEMS) s.tpb /= 2;
            }
        }
    }
    const double bin = dt_bytes(p.stages[a].in_dtype);
    s.bytes_per_px = bin + 4.0 + (ht > 0 && !s.streaming ? bin * ht / s.tpb : 0.0);
    // checkpointed IIRs: a first pass reads the input once more and writes each IIR's
    // double state at every run boundary, which the work items read back
    if (s.ckpt) s.bytes_per_px += bin + 16.0 * n_ck / s.tpb;
    s.cost = s.bytes_per_px * P * p.T;
    if (temporal && items > 0.0 && items < G_FILL_ITEMS) s.cost *= G_FILL_ITEMS / items;
    return s;
}

double partition_dp(const double* cost, int n, std::vector<int>& seg_last)
{
    // best[e]: optimum over stages 0..e-1; key (cost, groups, cut list)
    std::vector<double> best(n + 1, kInf);
    std::vector<int> groups(n + 1, 0);
    std::vector<std::vector<int>> cuts(n + 1);
    best[0] = 0.0;
    for (int e = 1; e <= n; ++e) {
        for (int a = 0; a < e; ++a) {  // last group a..e-1
            const double c = cost[(size_t)a * n + (e - 1)];
            if (!(best[a] < kInf) || !(c < kInf)) continue;
            const double tot = best[a] + c;
            const int g = groups[a] + 1;
            std::vector<int> cl = cuts[a];
            if (a > 0) cl.push_back(a - 1);
            bool better;
            if (!(best[e] < kInf)) better = true;
            else if (tot != best[e]) better = tot < best[e];
            else if (g != groups[e]) better = g < groups[e];
            else better = cl > cuts[e];  // later cuts win
            if (better) {
                best[e] = tot;
                groups[e] = g;
                cuts[e] = cl;
            }
        }
    }
    seg_last.clear();
    if (!(best[n] < kInf)) return kInf;
    seg_last = cuts[n];
    seg_last.push_back(n - 1);
    return best[n];
}

fz_plan* plan_for_size(const fz_plan& base, int W, int H, int T)
{
    fz_plan* p = new fz_plan();
    p->stages = base.stages;
    p->n = base.n;
    p->chain = base.chain;
    p->offset = base.offset;
    p->generic = base.generic;
    p->gweights = base.gweights;
    p->gwoff = base.gwoff;
    p->W = W;
    p->H = H;
    p->T = T;
    p->lds_budget = base.lds_budget;
    p->prm = base.prm;
    p->has_nms = base.has_nms;
    p->req_w = base.req_w;
    p->req_h = base.req_h;
    p->req_tpb = base.req_tpb;
    p->req_engine = base.req_engine;
    p->total = 0.0;
    for (const Segment& g : base.segs) {
        // keep each group's kernel family and tile; band / frame run re-chosen for the size
        const int eng = g.engine == FZ_ENGINE_TILE ? FZ_ENGINE_TILE : p->req_engine;
        const int rw = g.engine == FZ_ENGINE_TILE ? g.tile_w : 0;
        const int rh = g.engine == FZ_ENGINE_TILE ? g.tile_h : p->req_h;
        Segment s = price_group(*p, g.first, g.last, rw, rh, p->req_tpb, eng);
        if (!(s.cost < kInf)) {
            delete p;
            return nullptr;
        }
        p->total += s.cost;
        p->segs.push_back(s);
    }
    return p;
}

}  // namespace fz

fz_plan::~fz_plan() { fz::release_batch(*this); }

namespace fz {

// Generic stages: one channel, f32 out, u8 or f32 into the first stage and
// f32 into the others, radii in [0, G_MAX_R], finite stencil weights, a known
// point kind with finite parameters.
static fz_status validate_generic(const fz_stage* stages, int n)
{
    for (int i = 0; i < n; ++i) {
        const fz_stage& s = stages[i];
        const std::string where = "stage " + std::to_string(i) + ": ";
        if (s.in_ch != 1 || s.out_ch != 1 || s.out_dtype != FZ_F32)
            return fail(FZ_E_INVALID, where + "generic stages have one channel and f32 output");
        if (!(s.in_dtype == FZ_F32 || (i == 0 && s.in_dtype == FZ_U8)))
            return fail(FZ_E_INVALID, where + "input must be f32 (u8 allowed for the first stage)");
        if (s.dep < FZ_DEP_TT || s.dep > FZ_DEP_KK) return fail(FZ_E_INVALID, where + "bad dependence type");
        if (s.op == FZ_OP_IIR) {
            if (s.rx != 0 || s.ry != 0 || s.rt != -1)
                return fail(FZ_E_INVALID, where + "an IIR stage has radius 0 and reads every earlier frame (rt = -1)");
            if (!(s.param[0] > 0.0f && s.param[0] <= 1.0f))
                return fail(FZ_E_INVALID, where + "the IIR coefficient a must lie in (0, 1]");
            continue;
        }
        if (s.rt != 0 && !(s.op == FZ_OP_STENCIL && s.rt > 0 && s.rt <= G_MAX_RT))
            return fail(FZ_E_INVALID, where + "only a stencil may look back, at most " + std::to_string(G_MAX_RT) +
                                          " frames");
        if (s.op == FZ_OP_POINT) {
            const float k = s.param[0];
            if (s.rx != 0 || s.ry != 0) return fail(FZ_E_INVALID, where + "a point stage has radius 0");
            if (!(k >= 0.0f && k <= (float)FZ_POINT_CLAMP) || k != (float)(int)k)
                return fail(FZ_E_INVALID, where + "unknown point kind");
            if (!std::isfinite(s.param[1]) || !std::isfinite(s.param[2]))
                return fail(FZ_E_INVALID, where + "point parameters must be finite");
            if ((int)k == FZ_POINT_CLAMP && !(s.param[1] <= s.param[2]))
                return fail(FZ_E_INVALID, where + "clamp needs a <= b");
            continue;
        }
        if (s.rx < 0 || s.ry < 0 || s.rx > G_MAX_R || s.ry > G_MAX_R)
            return fail(FZ_E_INVALID, where + "window radii must be in [0, " + std::to_string(G_MAX_R) + "]");
        if ((s.rx > 0 || s.ry > 0) && s.dep == FZ_DEP_TT)
            return fail(FZ_E_INVALID, where + "a window stage cannot have a thread-to-thread dependence");
        if (s.op == FZ_OP_STENCIL) {
            if (!s.weights) return fail(FZ_E_INVALID, where + "stencil without weights");
            for (int q = 0; q < (2 * s.rx + 1) * (2 * s.ry + 1) * (s.rt + 1); ++q)
                if (!std::isfinite(s.weights[q])) return fail(FZ_E_INVALID, where + "stencil weights must be finite");
        }
    }
    return FZ_OK;
}

}  // namespace fz

using namespace fz;

extern "C" {

const char* fz_last_error(void) { return g_err.c_str(); }

const char* fz_version(void) { return "fz 0.1 gfx950"; }

fz_status fz_stage_describe(int32_t op, fz_stage* out)
{
    if (!out) return fail(FZ_E_INVALID, "fz_stage_describe: null output");
    const OpInfo o = op_info(op);
    if (o.op == 0) return fail(FZ_E_INVALID, "fz_stage_describe: unknown op " + std::to_string(op));
    memset(out, 0, sizeof(*out));
    out->op = op;
    out->rx = out->ry = o.r;
    out->rt = o.rt;
    out->in_ch = o.in_ch;
    out->out_ch = o.out_ch;
    out->in_dtype = o.in_dt;
    out->out_dtype = o.out_dt;
    out->dep = o.dep;
    if (op == FZ_OP_GAUSS5) out->param[0] = 1.0f;
    if (op == FZ_OP_HARRIS) out->param[0] = 0.04f;
    if (op == FZ_OP_THRESHOLD) out->param[0] = 1.0e8f;
    if (op == FZ_OP_STENCIL || op == FZ_OP_BOX) out->rx = out->ry = 1;
    if (op == FZ_OP_IIR) out->param[0] = 0.5f;
    if (op == FZ_OP_POINT) {
        out->param[0] = (float)FZ_POINT_AFFINE;
        out->param[1] = 1.0f;
    }
    return FZ_OK;
}

fz_status fz_box_eq6(double beta, double dx, double dt, double* x, double* t)
{
    if (!x || !t) return fail(FZ_E_INVALID, "fz_box_eq6: null output");
    if (!(beta > 0.0) || !(dx >= 0.0) || !(dt >= 0.0) || !std::isfinite(beta) || !std::isfinite(dx) ||
        !std::isfinite(dt))
        return fail(FZ_E_INVALID, "fz_box_eq6: beta must be positive and the halos non-negative");
    eq6_box(beta, dx, dt, x, t);
    return FZ_OK;
}

fz_status fz_partition_min(const double* cost, int32_t n, int32_t* seg_last, int32_t* n_seg, double* total)
{
    if (!cost || !seg_last || !n_seg || !total) return fail(FZ_E_INVALID, "fz_partition_min: null pointer");
    if (n < 1 || n > 64) return fail(FZ_E_INVALID, "fz_partition_min: n must be in [1, 64]");
    std::vector<int> sl;
    *total = partition_dp(cost, n, sl);
    *n_seg = (int32_t)sl.size();
    for (size_t i = 0; i < sl.size(); ++i) seg_last[i] = sl[i];
    return FZ_OK;
}

fz_status fz_plan_chain(const fz_stage* stages, int32_t n, const fz_plan_opts* opts, fz_plan** out)
{
    if (!stages || !opts || !out) return fail(FZ_E_INVALID, "fz_plan_chain: null pointer");
    *out = nullptr;
    if (n <= 0 || n > 16) return fail(FZ_E_INVALID, "fz_plan_chain: n must be in [1, 16]");
    if (opts->width <= 0 || opts->height <= 0 || opts->frames <= 0)
        return fail(FZ_E_INVALID, "fz_plan_chain: width, height and frames must be positive");
    if ((int64_t)opts->width * opts->height > (int64_t)1 << 28)
        return fail(FZ_E_INVALID, "fz_plan_chain: frame larger than 2^28 pixels");
    if (opts->cost_model != FZ_COST_ANALYTIC && opts->cost_model != FZ_COST_LEARNED &&
        opts->cost_model != FZ_COST_MEASURED)
        return fail(FZ_E_INVALID, "fz_plan_chain: unknown cost model");
    if (opts->cost_model == FZ_COST_LEARNED && (!opts->cost_weights || opts->cost_n_features != COST_FEATURES))
        return fail(FZ_E_INVALID, "fz_plan_chain: the learned cost model needs weights for " +
                                      std::to_string(COST_FEATURES) + " features");
    if (opts->frames_per_block < 0) return fail(FZ_E_INVALID, "fz_plan_chain: negative frames_per_block");
    if (opts->engine < FZ_ENGINE_AUTO || opts->engine > FZ_ENGINE_JIT || opts->engine == FZ_ENGINE_STREAM)
        return fail(FZ_E_INVALID, "fz_plan_chain: unknown engine");
    if (opts->tile_w > 0 && opts->tile_h <= 0)
        return fail(FZ_E_INVALID, "fz_plan_chain: a tile width needs a tile height");
    if (opts->tile_w < 0 || opts->tile_h < 0) return fail(FZ_E_INVALID, "fz_plan_chain: negative tile size");

    int n_generic = 0;
    for (int i = 0; i < n; ++i) n_generic += is_generic_op(stages[i].op);
    if (n_generic > 0 && n_generic < n)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_chain: generic stages cannot be mixed with the fixed operations");
    const bool generic = n_generic == n;
    if (opts->engine == FZ_ENGINE_JIT && !generic)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_chain: generated kernels are made for generic stages only");
    if (generic) {
        fz_status st = validate_generic(stages, n);
        if (st != FZ_OK) return st;
        if (opts->cost_model == FZ_COST_LEARNED)
            for (int i = 0; i < n; ++i)
                if (stages[i].op == FZ_OP_IIR || stages[i].rt > 0)
                    return fail(FZ_E_UNSUPPORTED, "fz_plan_chain: the cost network was not trained on temporal "
                                                  "stages (IIR, stencils that look back); use analytic or measured "
                                                  "prices");
    }
    // validate the descriptors against the operation registry (Sec. IV access patterns)
    for (int i = 0; i < n && !generic; ++i) {
        const fz_stage& s = stages[i];
        const OpInfo o = op_info(s.op);
        if (o.op == 0) return fail(FZ_E_INVALID, "stage " + std::to_string(i) + ": unknown op");
        if (s.rx != o.r || s.ry != o.r || s.rt != o.rt || s.in_ch != o.in_ch || s.out_ch != o.out_ch ||
            s.in_dtype != o.in_dt || s.out_dtype != o.out_dt)
            return fail(FZ_E_INVALID, "stage " + std::to_string(i) + ": access pattern does not match its op");
        if (s.dep < FZ_DEP_TT || s.dep > FZ_DEP_KK)
            return fail(FZ_E_INVALID, "stage " + std::to_string(i) + ": bad dependence type");
        if (i > 0 && (stages[i - 1].out_ch != s.in_ch || stages[i - 1].out_dtype != s.in_dtype))
            return fail(FZ_E_INVALID, "stage " + std::to_string(i) + ": input does not match the previous output");
    }
    // locate the chain among the compiled sequences
    int chain = -1, offset = generic ? 0 : -1;
    for (int c = 0; c < N_CHAINS && chain < 0 && !generic; ++c)
        for (int o = 0; o + n <= chain_len(c); ++o) {
            bool ok = true;
            for (int i = 0; i < n && ok; ++i) ok = chain_op(c, o + i) == stages[i].op;
            if (ok) {
                chain = c;
                offset = o;
                break;
            }
        }
    if (chain < 0 && !generic)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_chain: stage sequence is not one the kernels are built for");

    fz_plan* p = new fz_plan();
    p->stages.assign(stages, stages + n);
    p->n = n;
    p->generic = generic;
    if (generic) {
        // the plan keeps its own copy of the stencil weights
        p->gwoff.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            p->gwoff[i] = (int)p->gweights.size();
            if (stages[i].op == FZ_OP_STENCIL)
                p->gweights.insert(p->gweights.end(), stages[i].weights,
                                   stages[i].weights +
                                       (2 * stages[i].rx + 1) * (2 * stages[i].ry + 1) * (stages[i].rt + 1));
        }
    }
    for (fz_stage& st : p->stages) st.weights = nullptr;
    p->chain = chain;
    p->offset = offset;
    p->W = opts->width;
    p->H = opts->height;
    p->T = opts->frames;
    p->lds_budget = opts->lds_budget_bytes > 0 ? opts->lds_budget_bytes : 163840;
    for (int i = 0; i < n; ++i) {
        const fz_stage& s = stages[i];
        if (s.op == FZ_OP_GAUSS5) {
            if (!(s.param[0] > 0.0f)) {
                delete p;
                return fail(FZ_E_INVALID, "gauss5: sigma must be positive");
            }
            p->prm.sigma = s.param[0];
        }
        if (s.op == FZ_OP_HARRIS) p->prm.k = s.param[0];
        if (s.op == FZ_OP_THRESHOLD) p->prm.thr = s.param[0];
        if (s.op == FZ_OP_NMS3) p->has_nms = true;
    }
    {
        // sampled Gaussian weights, normalised in double, rounded once to FP32
        double w[3], sum = 0.0;
        const double sg = p->prm.sigma;
        for (int i = 0; i < 3; ++i) w[i] = exp(-(double)(i * i) / (2.0 * sg * sg));
        sum = w[0] + 2.0 * w[1] + 2.0 * w[2];
        for (int i = 0; i < 3; ++i) p->prm.gw[i] = (float)(w[i] / sum);
    }
    // a requested band or frame run that some row group cannot run is refused,
    // not replaced by another shape
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            const Segment s = price_group(*p, a, b, opts->tile_w, opts->tile_h, opts->frames_per_block, opts->engine);
            if (s.refused == 2) {
                delete p;
                return fail(FZ_E_UNSUPPORTED, "requested frame run of " + std::to_string(opts->frames_per_block) +
                                                  " frames: group " + std::to_string(a) + ".." + std::to_string(b) +
                                                  " holds an IIR, whose work items march every frame of the clip");
            }
            if (s.refused) {
                delete p;
                return fail(FZ_E_UNSUPPORTED, "requested band of " + std::to_string(opts->tile_h) +
                                                  " rows: the row kernel of group " + std::to_string(a) + ".." +
                                                  std::to_string(b) + " keeps at most " +
                                                  std::to_string(ROW_DIFF_MAX_BAND) +
                                                  " rows per band when it ends in the frame difference");
            }
        }
    // a stage that cannot run even alone makes the chain infeasible
    for (int i = 0; i < n; ++i) {
        Segment s = price_group(*p, i, i, opts->tile_w, opts->tile_h, opts->frames_per_block, opts->engine);
        if (!(s.cost < kInf)) {
            delete p;
            if (opts->tile_w > 0)
                return fail(FZ_E_UNSUPPORTED, "requested tile is not compiled or does not fit the budget");
            return fail(FZ_E_LDS, "stage " + std::to_string(i) + " does not fit the on-chip budget");
        }
    }
    p->cost.assign((size_t)n * n, kInf);
    std::vector<std::vector<Segment>> segtab(n, std::vector<Segment>(n));
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            segtab[a][b] = opts->cost_model == FZ_COST_LEARNED
                               ? price_group_learned(*p, a, b, opts->cost_weights, opts->tile_w, opts->tile_h,
                                                     opts->frames_per_block, opts->engine)
                               : price_group(*p, a, b, opts->tile_w, opts->tile_h, opts->frames_per_block,
                                             opts->engine);
            p->cost[(size_t)a * n + b] = segtab[a][b].cost;
        }
    std::vector<int> seg_last;
    if (opts->partition == FZ_PART_OPTIMAL) {
        p->total = partition_dp(p->cost.data(), n, seg_last);
    } else if (opts->partition == FZ_PART_UNFUSED) {
        for (int i = 0; i < n; ++i) seg_last.push_back(i);
    } else if (opts->partition == FZ_PART_EXPLICIT) {
        if (opts->n_cuts < 0 || opts->n_cuts > n - 1 || (opts->n_cuts > 0 && !opts->cuts)) {
            delete p;
            return fail(FZ_E_INVALID, "explicit partition: bad cut list");
        }
        int prev = -1;
        for (int i = 0; i < opts->n_cuts; ++i) {
            const int c = opts->cuts[i];
            if (c <= prev || c > n - 2) {
                delete p;
                return fail(FZ_E_INVALID, "explicit partition: cuts must increase strictly within [0, n-2]");
            }
            seg_last.push_back(c);
            prev = c;
        }
        seg_last.push_back(n - 1);
    } else {
        delete p;
        return fail(FZ_E_INVALID, "unknown partition mode");
    }
    if (seg_last.empty()) {
        delete p;
        return fail(FZ_E_LDS, "no partition of the chain fits the on-chip budget");
    }
    double total = 0.0;
    int a = 0;
    for (int last : seg_last) {
        const Segment& s = segtab[a][last];
        if (!(s.cost < kInf)) {
            delete p;
            return fail(FZ_E_LDS, "group " + std::to_string(a) + ".." + std::to_string(last) +
                                      " is not allowed (kernel-to-kernel dependence or on-chip budget)");
        }
        p->segs.push_back(s);
        total += s.cost;
        a = last + 1;
    }
    p->total = total;
    for (const Segment& g : p->segs)
        if (g.engine == FZ_ENGINE_JIT) {
            const fz_status st = jit_prepare(*p, g);
            if (st != FZ_OK) {
                delete p;
                return st;
            }
        }
    p->req_w = opts->tile_w;
    p->req_h = opts->tile_h;
    p->req_tpb = opts->frames_per_block;
    p->req_engine = opts->engine;
    *out = p;
    return FZ_OK;
}

void fz_plan_destroy(fz_plan* plan) { delete plan; }

int32_t fz_plan_num_segments(const fz_plan* plan) { return plan ? (int32_t)plan->segs.size() : -1; }

fz_status fz_plan_segments(const fz_plan* plan, int32_t* seg_last, int32_t cap)
{
    if (!plan || !seg_last) return fail(FZ_E_INVALID, "fz_plan_segments: null pointer");
    if (cap < (int32_t)plan->segs.size()) return fail(FZ_E_INVALID, "fz_plan_segments: capacity too small");
    for (size_t i = 0; i < plan->segs.size(); ++i) seg_last[i] = plan->segs[i].last;
    return FZ_OK;
}

fz_status fz_plan_segment_info(const fz_plan* plan, int32_t i, fz_segment_info* out)
{
    if (!plan || !out) return fail(FZ_E_INVALID, "fz_plan_segment_info: null pointer");
    if (i < 0 || i >= (int32_t)plan->segs.size()) return fail(FZ_E_INVALID, "fz_plan_segment_info: bad index");
    const Segment& s = plan->segs[i];
    out->first = s.first;
    out->last = s.last;
    out->tile_w = s.tile_w;
    out->tile_h = s.tile_h;
    out->frames_per_block = s.tpb;
    out->halo = s.halo;
    out->halo_t = s.halo_t;
    out->lds_bytes = s.lds_bytes;
    out->streaming = s.streaming;
    out->engine = s.engine;
    out->bytes_per_px = s.bytes_per_px;
    out->cost = s.cost;
    return FZ_OK;
}

fz_status fz_plan_set_segment_config(fz_plan* plan, int32_t i, int32_t engine, int32_t tile_w, int32_t tile_h,
                                     int32_t frames_per_block)
{
    if (!plan) return fail(FZ_E_INVALID, "fz_plan_set_segment_config: null plan");
    if (i < 0 || i >= (int32_t)plan->segs.size()) return fail(FZ_E_INVALID, "fz_plan_set_segment_config: bad index");
    if (engine < FZ_ENGINE_AUTO || engine > FZ_ENGINE_JIT || engine == FZ_ENGINE_STREAM || tile_w < 0 || tile_h < 0 ||
        frames_per_block < 0)
        return fail(FZ_E_INVALID, "fz_plan_set_segment_config: bad configuration");
    if (engine == FZ_ENGINE_JIT) {
        if (!plan->generic)
            return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: generated kernels are for generic stages only");
        if (tile_w > 0) {
            bool ok = false;
            for (int t = 0; t < N_JIT_TILES; ++t) ok |= JIT_TILES[t][0] == tile_w && JIT_TILES[t][1] == tile_h;
            if (!ok) return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: not a generated-kernel tile");
        }
        const Segment& o = plan->segs[i];
        Segment s = price_group(*plan, o.first, o.last, tile_w, tile_h, frames_per_block, FZ_ENGINE_JIT);
        if (s.refused)
            return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: the group holds an IIR after a window stage, "
                                          "whose work items march every frame of the clip");
        if (!(s.cost < kInf)) return fail(FZ_E_LDS, "fz_plan_set_segment_config: configuration does not fit the budget");
        if (s.engine != FZ_ENGINE_JIT)
            return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: no generated kernel for this group");
        const fz_status st = jit_prepare(*plan, s);
        if (st != FZ_OK) return st;
        plan->total += s.cost - o.cost;
        plan->segs[i] = s;
        release_batch(*plan);
        return FZ_OK;
    }
    if (engine == FZ_ENGINE_TILE && tile_w > 0 && tile_h <= 0)
        return fail(FZ_E_INVALID, "fz_plan_set_segment_config: a tile width needs a tile height");
    if (engine == FZ_ENGINE_TILE && tile_w > 0) {
        bool compiled = false;
        for (int t = 0; t < N_TILES; ++t) compiled |= fz::tile_w(t) == tile_w && fz::tile_h(t) == tile_h;
        if (!compiled) return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: tile not compiled");
    }
    const Segment& old = plan->segs[i];
    Segment s = price_group(*plan, old.first, old.last, engine == FZ_ENGINE_TILE ? tile_w : 0, tile_h,
                            frames_per_block, engine);
    if (s.refused == 2)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: the group holds an IIR, whose work items march "
                                      "every frame of the clip (frames_per_block must be 0 or the clip length)");
    if (s.refused)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: a band of " + std::to_string(tile_h) +
                                          " rows is over the " + std::to_string(ROW_DIFF_MAX_BAND) +
                                          " the row kernel keeps when the group ends in the frame difference");
    if (!(s.cost < kInf)) return fail(FZ_E_LDS, "fz_plan_set_segment_config: configuration does not fit the budget");
    if (engine == FZ_ENGINE_ROW && s.engine != FZ_ENGINE_ROW)
        return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: the row engine does not apply to this group");
    if (engine == FZ_ENGINE_TILE && tile_w > 0 && (s.tile_w != tile_w || s.tile_h != tile_h))
        return fail(FZ_E_UNSUPPORTED, "fz_plan_set_segment_config: tile not compiled");
    plan->total += s.cost - old.cost;
    plan->segs[i] = s;
    release_batch(*plan);
    return FZ_OK;
}

int32_t fz_cost_n_features(void) { return COST_FEATURES; }

int32_t fz_plan_segment_features(const fz_plan* plan, int32_t i, float* out, int32_t cap)
{
    if (!plan || !out || i < 0 || i >= (int32_t)plan->segs.size() || cap < COST_FEATURES) {
        set_error("fz_plan_segment_features: bad argument");
        return -1;
    }
    group_features(*plan, plan->segs[i], out);
    return COST_FEATURES;
}

double fz_plan_cost(const fz_plan* plan) { return plan ? plan->total : kInf; }

fz_status fz_plan_group_cost(const fz_plan* plan, int32_t a, int32_t b, double* cost)
{
    if (!plan || !cost) return fail(FZ_E_INVALID, "fz_plan_group_cost: null pointer");
    if (a < 0 || b < a || b >= plan->n) return fail(FZ_E_INVALID, "fz_plan_group_cost: bad range");
    *cost = plan->cost[(size_t)a * plan->n + b];
    return FZ_OK;
}

size_t fz_workspace_bytes(const fz_plan* plan) { return plan ? workspace_bytes(*plan) : 0; }

size_t fz_measure_workspace_bytes(const fz_plan* plan) { return plan ? measure_workspace_bytes(*plan) : 0; }

fz_status fz_plan_measure(fz_plan* plan, const void* d_in, void* d_workspace, size_t ws_bytes, int32_t reps,
                          void* stream)
{
    if (!plan || !d_in) return fail(FZ_E_INVALID, "fz_plan_measure: null plan or input");
    if (reps < 1 || reps > 1000) return fail(FZ_E_INVALID, "fz_plan_measure: reps must be in [1, 1000]");
    return plan_measure(*plan, d_in, d_workspace, ws_bytes, reps, stream);
}

size_t fz_batch_workspace_bytes(const fz_plan* plan, const fz_clip* clips, int32_t n_clips)
{
    if (!plan || !clips || n_clips <= 0) return 0;
    return batch_workspace_bytes(*plan, clips, n_clips);
}

fz_status fz_run_batch(fz_plan* plan, const fz_clip* clips, int32_t n_clips, void* d_workspace, size_t ws_bytes,
                       void* stream)
{
    if (!plan || !clips) return fail(FZ_E_INVALID, "fz_run_batch: null plan or clip array");
    if (n_clips < 1 || n_clips > 1024) return fail(FZ_E_INVALID, "fz_run_batch: n_clips must be in [1, 1024]");
    for (int i = 0; i < n_clips; ++i) {
        const fz_clip& c = clips[i];
        const std::string where = "fz_run_batch: clip " + std::to_string(i) + ": ";
        if (!c.d_in || !c.d_out) return fail(FZ_E_INVALID, where + "null input or output");
        if (c.width <= 0 || c.height <= 0 || c.frames <= 0) return fail(FZ_E_INVALID, where + "bad size");
        if ((int64_t)c.width * c.height > (int64_t)1 << 28) return fail(FZ_E_INVALID, where + "frame too large");
        if (c.point_capacity > 0 && !c.d_points) return fail(FZ_E_INVALID, where + "capacity without a point buffer");
    }
    const size_t need = batch_workspace_bytes(*plan, clips, n_clips);
    if (need == (size_t)-1) return fail(FZ_E_LDS, "fz_run_batch: the partition does not fit some clip's size");
    if (need > 0 && (!d_workspace || ws_bytes < need))
        return fail(FZ_E_WORKSPACE, "fz_run_batch: workspace needs " + std::to_string(need) + " bytes");
    return run_batch(*plan, clips, n_clips, d_workspace, ws_bytes, stream);
}

fz_status fz_run_chain(const fz_plan* plan, const void* d_in, void* d_out, fz_point* d_points, uint32_t* d_point_count,
                       uint32_t point_capacity, void* d_workspace, size_t ws_bytes, void* stream)
{
    if (!plan || !d_in || !d_out) return fail(FZ_E_INVALID, "fz_run_chain: null plan or buffer");
    if (point_capacity > 0 && !d_points) return fail(FZ_E_INVALID, "fz_run_chain: capacity without a point buffer");
    const size_t need = workspace_bytes(*plan);
    if (need > 0 && (!d_workspace || ws_bytes < need))
        return fail(FZ_E_WORKSPACE, "fz_run_chain: workspace needs " + std::to_string(need) + " bytes");
    return run_plan(*plan, d_in, d_out, d_points, d_point_count, point_capacity, d_workspace, ws_bytes, stream);
}

}  // extern "C"
