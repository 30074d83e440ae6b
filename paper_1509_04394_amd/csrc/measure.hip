// Measured prices: the paper's group cost C_i is the group's execution time
// (Sec. VI-A, Fig. 5).  Every contiguous group of a plan is timed with HIP
// events in every kernel configuration it can run in, on the plan's own input
// and the chain's real intermediates, and the partition is re-solved by the
// exact DP over the least measured time of each group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "fz_internal.h"

namespace fz {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t stage_out_bytes(const fz_plan& p, int k)
{
    const fz_stage& st = p.stages[k];
    return (size_t)p.W * p.H * p.T * st.out_ch * dt_bytes(st.out_dtype);
}

// Three buffers as large as the largest stage output (the input of the groups
// being timed, the output they write, the next stage's input), a counter, and
// the IIR checkpoints of the largest candidate group.
static size_t group_ws(const fz_plan& p, const Segment& g) { return align256(ckpt_bytes(p, g)) + exchange_bytes(p, g); }

// The largest single-group workspace (IIR checkpoints, frame-boundary
// exchange) of any group the measurement may time.
static size_t measure_ckpt_bytes(const fz_plan& p)
{
    size_t ck = 0;
    for (int a = 0; a < p.n; ++a)
        for (int b = a; b < p.n; ++b) {
            ck = std::max(ck, group_ws(p, price_group(p, a, b, 0, 0, 0, FZ_ENGINE_AUTO)));
            for (int t = 0; t < N_TILES; ++t)
                ck = std::max(ck, group_ws(p, price_group(p, a, b, tile_w(t), tile_h(t), 0, FZ_ENGINE_TILE)));
        }
    return ck;
}

size_t measure_workspace_bytes(const fz_plan& p)
{
    size_t mx = 0;
    for (int k = 0; k < p.n; ++k) mx = std::max(mx, stage_out_bytes(p, k));
    return 3 * align256(mx) + 256 + measure_ckpt_bytes(p);
}

// A plan of the same chain and size whose only group is g.
static void single_group(fz_plan& sub, const fz_plan& p, const Segment& g)
{
    sub.stages = p.stages;
    sub.n = p.n;
    sub.chain = p.chain;
    sub.offset = p.offset;
    sub.generic = p.generic;
    sub.gweights = p.gweights;
    sub.gwoff = p.gwoff;
    sub.W = p.W;
    sub.H = p.H;
    sub.T = p.T;
    sub.lds_budget = p.lds_budget;
    sub.prm = p.prm;
    sub.has_nms = false;
    for (int j = g.first; j <= g.last; ++j) sub.has_nms |= p.stages[j].op == FZ_OP_NMS3;
    sub.segs.assign(1, g);
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Median time in microseconds of `reps` runs of group g (after one untimed run).
static fz_status time_group(const fz_plan& p, const Segment& g, const void* in, void* out, uint32_t* cnt, int reps,
                            hipStream_t s, const EventPair& ev, void* ck, size_t ck_bytes, double* us)
{
    fz_plan sub;
    single_group(sub, p, g);
    std::vector<float> ms;
    for (int r = 0; r <= reps; ++r) {
        hipError_t e = hipEventRecord(ev.a, s);
        if (e != hipSuccess) return fail(FZ_E_HIP, std::string("measure: event record: ") + hipGetErrorString(e));
        fz_status st = run_plan(sub, in, out, nullptr, cnt, 0u, ck, ck_bytes, s);
        if (st != FZ_OK) return st;
        e = hipEventRecord(ev.b, s);
        if (e == hipSuccess) e = hipEventSynchronize(ev.b);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.a, ev.b);
        if (e != hipSuccess) return fail(FZ_E_HIP, std::string("measure: timing: ") + hipGetErrorString(e));
        if (r > 0) ms.push_back(t);
    }
    std::sort(ms.begin(), ms.end());
    *us = 1e3 * (double)ms[ms.size() / 2];
    return FZ_OK;
}

fz_status plan_measure(fz_plan& p, const void* d_in, void* ws, size_t ws_bytes, int reps, void* stream)
{
    const double inf = std::numeric_limits<double>::infinity();
    const size_t need = measure_workspace_bytes(p);
    if (!ws || ws_bytes < need)
        return fail(FZ_E_WORKSPACE, "fz_plan_measure: workspace needs " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    const size_t ckb = measure_ckpt_bytes(p);
    const size_t slot = (need - 256 - ckb) / 3;
    char* buf[3] = {(char*)ws, (char*)ws + slot, (char*)ws + 2 * slot};
    uint32_t* cnt = (uint32_t*)((char*)ws + 3 * slot);
    void* ck = ckb ? (void*)((char*)ws + 3 * slot + 256) : nullptr;
    EventPair ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("measure: event create: ") + hipGetErrorString(e));

    const int n = p.n;
    std::vector<double> cost((size_t)n * n, inf);
    std::vector<Segment> best((size_t)n * n);
    const void* cur = d_in;  // input of stage a
    int cur_buf = -1;
    for (int a = 0; a < n; ++a) {
        // the two buffers that do not hold the current input: group outputs
        // (discarded) and stage a's own output (the next input)
        int other[2], k = 0;
        for (int q = 0; q < 3; ++q)
            if (q != cur_buf && k < 2) other[k++] = q;
        const int out_buf = other[0], next_buf = other[1];
        for (int b = a; b < n; ++b) {
            std::vector<Segment> cands;
            cands.push_back(price_group(p, a, b, 0, 0, 0, FZ_ENGINE_AUTO));
            for (int t = 0; t < N_TILES; ++t) cands.push_back(price_group(p, a, b, tile_w(t), tile_h(t), 0, FZ_ENGINE_TILE));
            std::vector<std::pair<int, int>> seen;  // (engine, tile) already timed
            for (Segment& g : cands) {
                if (!(g.cost < inf)) continue;
                const std::pair<int, int> key(g.engine, g.engine == FZ_ENGINE_TILE ? g.tile : -1);
                if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
                seen.push_back(key);
                double us = 0.0;
                fz_status st = time_group(p, g, cur, buf[out_buf], cnt, reps, s, ev, ck, ckb, &us);
                if (st != FZ_OK) return st;
                if (us < cost[(size_t)a * n + b]) {
                    cost[(size_t)a * n + b] = us;
                    g.cost = us;
                    best[(size_t)a * n + b] = g;
                }
            }
        }
        if (a + 1 < n) {  // stage a alone gives the next stage's real input
            if (!(cost[(size_t)a * n + a] < inf))  // (best[] holds a timed configuration only where cost is finite)
                return fail(FZ_E_LDS, "fz_plan_measure: stage " + std::to_string(a) + " cannot run");
            const Segment g1 = best[(size_t)a * n + a];
            fz_plan sub;
            single_group(sub, p, g1);
            fz_status st = run_plan(sub, cur, buf[next_buf], nullptr, cnt, 0u, ck, ckb, s);
            if (st != FZ_OK) return st;
            cur = buf[next_buf];
            cur_buf = next_buf;
        }
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("measure: ") + hipGetErrorString(e));

    std::vector<int> seg_last;
    const double total = partition_dp(cost.data(), n, seg_last);
    if (seg_last.empty()) return fail(FZ_E_LDS, "fz_plan_measure: no partition can run");
    p.cost = cost;
    p.segs.clear();
    int a = 0;
    for (int last : seg_last) {
        p.segs.push_back(best[(size_t)a * n + last]);
        a = last + 1;
    }
    p.total = total;
    release_batch(p);
    return FZ_OK;
}

}  // namespace fz
