// Device-side execution of a plan: the groups run in order on the caller's
// stream; each group's output lands in the workspace (or the caller's output
// for the last group) and is the next group's input (Sec. VI: fused kernels
// execute in a sequence consistent with the original order).
#include <hip/hip_runtime.h>

#include <string>

#include "fz_internal.h"
#include "rowfuse.h"
#include "tables.h"
#include "tables_rowgen.h"

namespace fz {

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t group_out_bytes(const fz_plan& p, const Segment& s)
{
    const fz_stage& st = p.stages[s.last];
    return (size_t)p.W * p.H * p.T * st.out_ch * dt_bytes(st.out_dtype);
}

// Two ping-pong slots, each as large as the largest intermediate, then the
// largest group's IIR checkpoints (generic groups run in frame runs shorter
// than the clip).
static size_t slots_bytes(const fz_plan& p)
{
    size_t mx = 0;
    for (size_t i = 0; i + 1 < p.segs.size(); ++i) mx = std::max(mx, group_out_bytes(p, p.segs[i]));
    if (mx == 0) return 0;
    return (p.segs.size() > 2 ? 2 : 1) * align256(mx);
}

// Frame-boundary exchange of a frame-difference group of the Harris row
// kernel (0 for every other group).
size_t exchange_bytes(const fz_plan& p, const Segment& g)
{
    if (p.generic || g.engine != FZ_ENGINE_ROW || g.row_gen || g.clast != 8) return 0;
    return row_exchange_bytes(g.nstrips, g.nbands, g.nchunks, g.tile_h, g.row_k);
}

// Layout: the intermediate slots, the IIR checkpoints, the row kernel's
// frame-boundary exchange.
size_t workspace_bytes(const fz_plan& p)
{
    size_t ck = 0, xb = 0;
    for (const Segment& g : p.segs) {
        ck = std::max(ck, ckpt_bytes(p, g));
        xb = std::max(xb, exchange_bytes(p, g));
    }
    return slots_bytes(p) + align256(ck) + xb;
}

fz_status run_plan(const fz_plan& p, const void* d_in, void* d_out, fz_point* d_points, uint32_t* d_count,
                   uint32_t cap, void* d_ws, size_t ws_bytes, void* stream)
{
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    hipStream_t s = (hipStream_t)stream;
    const size_t slot = p.segs.size() > 1 ? align256(slots_bytes(p) / (p.segs.size() > 2 ? 2 : 1)) : 0;
    void* ckpt = d_ws ? (void*)((char*)d_ws + slots_bytes(p)) : nullptr;
    size_t ck = 0;
    for (const Segment& g : p.segs) ck = std::max(ck, ckpt_bytes(p, g));
    char* xch = d_ws ? (char*)d_ws + slots_bytes(p) + align256(ck) : nullptr;
    if (d_count && p.has_nms) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, d_count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(FZ_E_HIP, std::string("zeroing the point count: ") + hipGetErrorString(e));
    }
    const void* cur_in = d_in;
    for (size_t i = 0; i < p.segs.size(); ++i) {
        const Segment& g = p.segs[i];
        SegParams sp{};
        sp.in = cur_in;
        sp.out = (i + 1 == p.segs.size()) ? d_out : (void*)((char*)d_ws + (i % 2) * slot);
        sp.W = p.W;
        sp.H = p.H;
        sp.T = p.T;
        sp.tpb = g.tpb;
        sp.gw.w0 = p.prm.gw[0];
        sp.gw.w1 = p.prm.gw[1];
        sp.gw.w2 = p.prm.gw[2];
        sp.k = p.prm.k;
        sp.thr = p.prm.thr;
        sp.points = d_points;
        sp.count = d_count;
        sp.cap = d_points ? cap : 0u;
        bool group_has_nms = false;
        for (int j = g.first; j <= g.last; ++j) group_has_nms |= p.stages[j].op == FZ_OP_NMS3;
        if (!group_has_nms) sp.count = nullptr;
        hipError_t e;
        if (p.generic) {
            e = (hipError_t)launch_generic(p, g, sp.in, sp.out, ckpt, s);
        } else if (g.engine == FZ_ENGINE_ROW) {
            RowParams rp{};
            rp.sp = sp;
            rp.nstrips = g.nstrips;
            rp.nbands = g.nbands;
            rp.nchunks = g.nchunks;
            rp.total = g.nstrips * g.nbands * g.nchunks;
            rp.band_h = g.tile_h;
            rp.tt = g.tpb;
            if (g.row_gen) {
                rp.strip_step = 64 * g.row_k - 2 * g.halo;
                RowGenFn fn = lookup_rowgen(p.chain, g.cfirst, g.clast);
                if (!fn) return fail(FZ_E_UNSUPPORTED, "no row kernel compiled for this group");
                e = fn(rp, s);
            } else {
                rp.strip_step = 64 * g.row_k - 2 * ROW_HX;
                const size_t xb = exchange_bytes(p, g);
                if (xb > 0) {
                    if (!xch || ws_bytes < workspace_bytes(p))
                        return fail(FZ_E_WORKSPACE, "the frame-difference row group needs the exchange workspace");
                    const size_t nb = (size_t)row_boundaries(g.nstrips, g.nbands, g.nchunks);
                    rp.xmask = (uint64_t*)xch;
                    rp.xcount = (uint32_t*)(xch + ((2 * nb * g.tile_h * g.row_k * 8 + 255) & ~(size_t)255));
                }
                e = launch_rowfuse(rp, g.row_k, g.cfirst == 0, g.clast == 8, s);
            }
        } else {
            LaunchFn fn = lookup(p.chain, g.cfirst, g.clast);
            if (!fn) return fail(FZ_E_UNSUPPORTED, "no kernel compiled for this group");
            e = fn(sp, g.tile, s);
        }
        if (e != hipSuccess)
            return fail(FZ_E_HIP, "launching group " + std::to_string(g.first) + ".." + std::to_string(g.last) +
                                      ": " + hipGetErrorString(e));
        cur_in = sp.out;
    }
    return FZ_OK;
}

}  // namespace fz
