// Batches of clips: one persistent row-kernel launch over every clip's work
// items when the plan is a single group the row kernel implements, otherwise
// the clips' groups one clip after another; either way captured once into a
// HIP graph and replayed while the clip set is unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <string>

#include "fz_internal.h"
#include "rowfuse.h"

namespace fz {

static bool batch_persistent(const fz_plan& p, const fz_clip* clips, int n)
{
    if (p.segs.size() != 1) return false;
    const Segment& g = p.segs[0];
    if (!row_group(p.chain, g.cfirst, g.clast) || g.engine != FZ_ENGINE_ROW || g.row_gen) return false;
    for (int i = 0; i < n; ++i)
        if (clips[i].width < 128 || clips[i].height < 8) return false;
    return true;
}

constexpr size_t QUEUE_STRIDE = 256;  // one queue counter per launch, 256 bytes apart

size_t batch_workspace_bytes(const fz_plan& p, const fz_clip* clips, int n)
{
    if (batch_persistent(p, clips, n)) return QUEUE_STRIDE * ((n + FZ_BATCH_MAX - 1) / FZ_BATCH_MAX);
    size_t mx = 0;
    for (int i = 0; i < n; ++i) {
        std::unique_ptr<fz_plan> cp(plan_for_size(p, clips[i].width, clips[i].height, clips[i].frames));
        if (!cp) return (size_t)-1;
        mx = std::max(mx, workspace_bytes(*cp));
    }
    return mx;
}

static void release_graph(fz_plan& p)
{
    if (p.batch_exec) (void)hipGraphExecDestroy((hipGraphExec_t)p.batch_exec);
    if (p.batch_graph) (void)hipGraphDestroy((hipGraph_t)p.batch_graph);
    p.batch_exec = nullptr;
    p.batch_graph = nullptr;
    p.batch_key.clear();
}

void release_batch(fz_plan& p)
{
    release_graph(p);
    if (p.capture_stream) (void)hipStreamDestroy((hipStream_t)p.capture_stream);
    p.capture_stream = nullptr;
}

static std::vector<uint64_t> batch_key(const fz_clip* clips, int n, void* ws, size_t ws_bytes)
{
    std::vector<uint64_t> k;
    k.reserve(8 * n + 3);
    k.push_back((uint64_t)n);
    k.push_back((uint64_t)(uintptr_t)ws);
    k.push_back((uint64_t)ws_bytes);
    for (int i = 0; i < n; ++i) {
        const fz_clip& c = clips[i];
        k.push_back((uint64_t)(uintptr_t)c.d_in);
        k.push_back((uint64_t)(uintptr_t)c.d_out);
        k.push_back((uint64_t)(uintptr_t)c.d_points);
        k.push_back((uint64_t)(uintptr_t)c.d_point_count);
        k.push_back((uint64_t)c.point_capacity);
        k.push_back((uint64_t)(uint32_t)c.width);
        k.push_back((uint64_t)(uint32_t)c.height);
        k.push_back((uint64_t)(uint32_t)c.frames);
    }
    return k;
}

// Enqueue the batch on stream s (being captured).
static fz_status enqueue_batch(const fz_plan& p, const fz_clip* clips, int n, void* ws, size_t ws_bytes, hipStream_t s,
                               int cus)
{
    if (batch_persistent(p, clips, n)) {
        const Segment& g = p.segs[0];
        const bool rgb = g.cfirst == 0, diff = g.clast == 8;
        int bpc = rowfuse_batch_blocks_per_cu(2, rgb, diff);
        if (bpc < 1) bpc = 1;
        for (int c0 = 0; c0 < n; c0 += FZ_BATCH_MAX) {
            const int m = std::min(n - c0, FZ_BATCH_MAX);
            BatchParams bp{};
            bp.gw.w0 = p.prm.gw[0];
            bp.gw.w1 = p.prm.gw[1];
            bp.gw.w2 = p.prm.gw[2];
            bp.k = p.prm.k;
            bp.thr = p.prm.thr;
            bp.n_clips = m;
            bp.queue = (uint32_t*)((char*)ws + QUEUE_STRIDE * (c0 / FZ_BATCH_MAX));
            int items = 0;
            for (int i = 0; i < m; ++i) {
                const fz_clip& c = clips[c0 + i];
                BatchClip& b = bp.clip[i];
                b.in = c.d_in;
                b.out = c.d_out;
                b.points = c.d_points;
                b.count = p.has_nms ? c.d_point_count : nullptr;
                b.cap = c.d_points ? c.point_capacity : 0u;
                b.W = c.width;
                b.H = c.height;
                b.T = c.frames;
                b.nstrips = row_strips(c.width, 2);
                b.nbands = (c.height + BATCH_BAND_H - 1) / BATCH_BAND_H;
                b.nchunks = (c.frames + BATCH_TT - 1) / BATCH_TT;
                b.item_begin = items;
                items += b.nstrips * b.nbands * b.nchunks;
            }
            bp.total = items;
            const int blocks = std::max(1, std::min((items + ROW_WAVES - 1) / ROW_WAVES, cus * bpc));
            hipError_t e = launch_rowfuse_batch(bp, 2, rgb, diff, blocks, s);
            if (e != hipSuccess) return fail(FZ_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
        }
        return FZ_OK;
    }
    for (int i = 0; i < n; ++i) {
        const fz_clip& c = clips[i];
        std::unique_ptr<fz_plan> cp(plan_for_size(p, c.width, c.height, c.frames));
        if (!cp) return fail(FZ_E_LDS, "batch: the partition does not fit clip " + std::to_string(i));
        fz_status st = run_plan(*cp, c.d_in, c.d_out, c.d_points, c.d_point_count, c.point_capacity, ws, ws_bytes, s);
        if (st != FZ_OK) return st;
    }
    return FZ_OK;
}

fz_status run_batch(fz_plan& p, const fz_clip* clips, int n, void* ws, size_t ws_bytes, void* stream)
{
    hipStream_t user = (hipStream_t)stream;
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    std::vector<uint64_t> key = batch_key(clips, n, ws, ws_bytes);
    if (p.batch_exec && key == p.batch_key) {
        hipError_t e = hipGraphLaunch((hipGraphExec_t)p.batch_exec, user);
        if (e != hipSuccess) return fail(FZ_E_HIP, std::string("batch graph launch: ") + hipGetErrorString(e));
        return FZ_OK;
    }
    release_graph(p);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("device query: ") + hipGetErrorString(e));
    if (!p.capture_stream) {
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(FZ_E_HIP, std::string("capture stream: ") + hipGetErrorString(e));
        p.capture_stream = cs;
    }
    hipStream_t cs = (hipStream_t)p.capture_stream;
    // generated kernels are compiled and their modules loaded before the capture
    for (int i = 0; i < n; ++i) {
        bool any = false;
        for (const Segment& g : p.segs) any |= g.engine == FZ_ENGINE_JIT || p.req_engine == FZ_ENGINE_JIT;
        if (!any) break;
        std::unique_ptr<fz_plan> cp(plan_for_size(p, clips[i].width, clips[i].height, clips[i].frames));
        if (!cp) return fail(FZ_E_LDS, "batch: the partition does not fit clip " + std::to_string(i));
        for (const Segment& g : cp->segs)
            if (g.engine == FZ_ENGINE_JIT && (e = (hipError_t)jit_load(*cp, g)) != hipSuccess)
                return fail(FZ_E_HIP, std::string("batch: loading a generated kernel: ") + hipGetErrorString(e));
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    fz_status st = enqueue_batch(p, clips, n, ws, ws_bytes, cs, cus);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (st != FZ_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("end capture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(FZ_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    p.batch_graph = g;
    p.batch_exec = x;
    p.batch_key = key;
    e = hipGraphLaunch(x, user);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("batch graph launch: ") + hipGetErrorString(e));
    return FZ_OK;
}

}  // namespace fz
