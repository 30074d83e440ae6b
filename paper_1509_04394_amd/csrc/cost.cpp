// Learned group prices: features of a fused group in a given kernel
// configuration, and the cost network's forward pass on the host for planning
// (the same network the GPU kernels train; parameter layout in mlp.hip).
#include <math.h>

#include <algorithm>
#include <limits>
#include <vector>

#include "fz_internal.h"
#include "generic.h"
#include "rowgeom.h"

namespace fz {

static double log2p(double v) { return log2(v > 0 ? v : 1e-30); }

// Features of group g of plan p (all O(1) by construction; no normalisation
// statistics are needed).
void group_features(const fz_plan& p, const Segment& g, float* f)
{
    const int ch = p.chain, A = g.cfirst, B = g.clast;
    int nwin = 0, ops = 0, bytes_in, bytes_out;
    if (p.generic) {
        for (int j = g.first; j <= g.last; ++j) {
            const fz_stage& s = p.stages[j];
            const int kind = g_kind(s.op);
            nwin += g_is_window(kind);
            ops += generic_ops(kind, s.rx, s.ry, (int)s.param[0], s.rt > 0 ? s.rt : 0);
        }
        bytes_in = dt_bytes(p.stages[g.first].in_dtype);
        bytes_out = 4;
    } else {
        for (int j = A; j <= B; ++j) {
            const OpInfo o = op_info(chain_op(ch, j));
            nwin += o.r > 0;
            ops += o.ops_per_px;
        }
        const OpInfo oa = op_info(chain_op(ch, A)), ob = op_info(chain_op(ch, B));
        bytes_in = oa.in_ch * dt_bytes(oa.in_dt);
        bytes_out = ob.out_ch * dt_bytes(ob.out_dt);
    }
    const double W = p.W, H = p.H, T = p.T;
    double recompute = 1.0;
    if (g.engine == FZ_ENGINE_TILE && g.tile_w > 0)
        recompute = (double)(g.tile_w + 2 * g.halo) * (g.tile_h + 2 * g.halo_y) / ((double)g.tile_w * g.tile_h);
    if (g.engine == FZ_ENGINE_ROW)
        recompute = (double)g.nstrips * 64 * g.row_k / W * (g.tile_h + 2.0 * g.halo) / g.tile_h;
    const double temporal = g.halo_t > 0 ? (g.tpb + (double)g.halo_t) / g.tpb : 1.0;
    int i = 0;
    f[i++] = (float)((B - A + 1) / 9.0);
    f[i++] = (float)(nwin / 4.0);
    f[i++] = (float)((g.halo + g.halo_y) / 12.0);
    f[i++] = (float)g.halo_t;
    f[i++] = (float)(bytes_in / 12.0);
    f[i++] = (float)(bytes_out / 12.0);
    f[i++] = (float)(ops / 73.0);
    f[i++] = g.engine == FZ_ENGINE_TILE ? 1.0f : 0.0f;
    f[i++] = g.engine == FZ_ENGINE_ROW ? 1.0f : 0.0f;
    f[i++] = g.engine == FZ_ENGINE_STREAM ? 1.0f : 0.0f;
    f[i++] = (float)(g.tile_w > 0 ? log2p(g.tile_w) / 8.0 : 0.0);
    f[i++] = (float)(g.tile_h > 0 ? log2p(g.tile_h) / 8.0 : 0.0);
    f[i++] = (float)(log2p(g.tpb + 1.0) / 6.0);
    f[i++] = (float)(g.lds_bytes / 65536.0);
    f[i++] = (float)(log2p(W * H) / 20.0);
    f[i++] = (float)(log2p(T) / 10.0);
    f[i++] = (float)log2p(recompute * temporal);
    f[i++] = (float)(log2p(W * H * T * ops) / 40.0);
    f[i++] = (g.engine == FZ_ENGINE_ROW && !g.row_gen) ? 1.0f : 0.0f;  // the Harris-chain row kernel
    f[i++] = p.generic ? 1.0f : 0.0f;                                     // the generic-stage kernels
}

// Forward pass of the cost network (parameter layout of mlp.hip).
double mlp_predict(const float* prm, const float* x)
{
    constexpr int F = COST_FEATURES, Hd = 64;
    const float* w1 = prm;
    const float* b1 = w1 + Hd * F;
    const float* w2 = b1 + Hd;
    const float* b2 = w2 + Hd * Hd;
    const float* w3 = b2 + Hd;
    const float* b3 = w3 + Hd;
    float h1[Hd], h2[Hd];
    for (int j = 0; j < Hd; ++j) {
        float a = b1[j];
        for (int k = 0; k < F; ++k) a = fmaf(w1[j * F + k], x[k], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < Hd; ++j) {
        float a = b2[j];
        for (int k = 0; k < Hd; ++k) a = fmaf(w2[j * Hd + k], h1[k], a);
        h2[j] = a > 0.0f ? a : 0.0f;
    }
    float y = b3[0];
    for (int k = 0; k < Hd; ++k) y = fmaf(w3[k], h2[k], y);
    return y;
}

// Learned price of group [a..b]: the configuration (engine, tile) with the
// least predicted time among those the requests allow; cost = predicted us.
Segment price_group_learned(const fz_plan& p, int a, int b, const float* prm, int req_w, int req_h, int req_tpb,
                            int req_engine)
{
    const double inf = std::numeric_limits<double>::infinity();
    Segment best{};
    best.cost = inf;
    std::vector<Segment> cands;
    if (req_w > 0 || req_engine != FZ_ENGINE_AUTO) {
        cands.push_back(price_group(p, a, b, req_w, req_h, req_tpb, req_engine));
    } else {
        cands.push_back(price_group(p, a, b, 0, req_h, req_tpb, FZ_ENGINE_AUTO));
        for (int t = 0; t < N_TILES; ++t)
            cands.push_back(price_group(p, a, b, tile_w(t), tile_h(t), req_tpb, FZ_ENGINE_TILE));
    }
    float x[COST_FEATURES];
    for (Segment& s : cands) {
        if (!(s.cost < inf)) continue;
        group_features(p, s, x);
        const double us = exp(mlp_predict(prm, x));
        if (us < best.cost) {
            best = s;
            best.cost = us;
        }
    }
    if (!(best.cost < inf)) best = cands[0];
    return best;
}

}  // namespace fz
