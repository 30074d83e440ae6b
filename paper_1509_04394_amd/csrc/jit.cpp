// Generated fused kernels for generic groups (the paper's future work,
// Sec. X: generating the fused kernel from the kernels' descriptions).
//
// The generic tile kernel interprets its group's stage list for every cell:
// a switch per point stage, loops over run-time radii, run-time box sizes.
// Here the group's kernel is written out as source text instead -- the stage
// list unrolled, every radius, box size and weight a compile-time constant,
// point operations inline -- compiled for gfx950 with hipRTC (on the host; no
// device needed), loaded per device on first use and cached by its source
// text for the life of the process.  The generated kernel keeps the tile
// kernel's structure (input box loaded once into LDS with the leading point
// stages applied, window stages from one LDS buffer into the other, the last
// one straight to global memory, five neighbouring cells per thread inside the
// frame, clamped reads on border tiles) and the same arithmetic in the same
// order, so its output equals the tile kernel's to the bit.  Groups with a
// temporal stage get the frame-marching kernel written out the same way
// (rings of earlier frames per stencil, IIR states, checkpoint restore).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "fz_internal.h"
#include "generic.h"

namespace fz {

// Output tiles the generated kernels may use (x by y).
const int JIT_TILES[N_JIT_TILES][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 16}, {64, 32}};

static std::string flit(float v)
{
    char b[64];
    snprintf(b, sizeof b, "%af", (double)v);  // hexadecimal: exact
    return b;
}

// One point stage applied to `v`, as an expression statement.
static std::string point_stmt(const fz_stage& s)
{
    const int k = (int)s.param[0];
    const std::string a = flit(s.param[1]), b = flit(s.param[2]);
    switch (k) {
    case FZ_POINT_AFFINE: return "v = fmaf(" + a + ", v, " + b + ");";
    case FZ_POINT_ABS: return "v = fabsf(v);";
    case FZ_POINT_SQUARE: return "v = v * v;";
    case FZ_POINT_SQRTABS: return "v = sqrtf(fabsf(v));";
    default: return "v = fminf(fmaxf(v, " + a + "), " + b + ");";
    }
}

static std::string jit_march_source(const fz_plan& p, const Segment& g);

std::string jit_source(const fz_plan& p, const Segment& g)
{
    {
        GStage st[G_MAX_STAGES];
        g_stage_list(p.stages.data(), g.first, g.last, st);
        if (g_temporal(st, g.last - g.first + 1)) return jit_march_source(p, g);
    }
    std::ostringstream o;
    const int TW = g.tile_w, TH = g.tile_h, HX = g.halo, HY = g.halo_y;
    const bool u8 = p.stages[g.first].in_dtype == FZ_U8;
    o << "#define GQ 5\n"
         "__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }\n"
         "extern \"C\" __global__ __launch_bounds__(256) void fz_jit(const "
      << (u8 ? "unsigned char" : "float")
      << "* __restrict__ in, float* __restrict__ out, int W, int H, int tiles_x, int tiles_y)\n{\n"
      << "    constexpr int TW = " << TW << ", TH = " << TH << ", HX = " << HX << ", HY = " << HY
      << ", RW = TW + 2 * HX, RH = TH + 2 * HY;\n";
    int nwin = 0;
    for (int j = g.first; j <= g.last; ++j) nwin += p.stages[j].op != FZ_OP_POINT;
    o << "    __shared__ float lds[" << generic_lds_bytes(TW, TH, HX, HY, nwin) / 4 << "];\n"
      << "    float* bufs[2] = {lds, lds + RW * RH};\n"
         // blocks dealt to XCDs round-robin: contiguous runs of tiles per XCD
         "    const int nb = gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;\n"
         "    int b = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + slot;\n"
         "    const int tx = b % tiles_x;\n    b /= tiles_x;\n    const int ty = b % tiles_y;\n"
         "    const int t = b / tiles_y;\n"
         "    const int ox = tx * TW - HX, oy = ty * TH - HY;\n"
         "    const size_t fbase = (size_t)t * W * H;\n"
         "    const bool interior = ox >= 0 && oy >= 0 && ox + RW <= W && oy + RH <= H;\n";
    // load with the leading point stages
    int j = g.first;
    o << "    for (int e = threadIdx.x; e < RW * RH; e += 256) {\n"
         "        const int ly = e / RW, lx = e - ly * RW;\n"
         "        const int gx = ox + lx, gy = oy + ly;\n"
         "        if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;\n"
         "        float v = (float)in[fbase + (size_t)gy * W + gx];\n";
    for (; j <= g.last && p.stages[j].op == FZ_OP_POINT; ++j) o << "        " << point_stmt(p.stages[j]) << "\n";
    o << "        bufs[0][e] = v;\n    }\n    __syncthreads();\n";
    int hx = HX, hy = HY, step = 0;
    while (j <= g.last) {
        const fz_stage& s = p.stages[j];
        int k = j + 1;
        while (k <= g.last && p.stages[k].op == FZ_OP_POINT) ++k;
        const bool last = k > g.last;
        const bool stencil = s.op == FZ_OP_STENCIL;
        const int ohx = hx - s.rx, ohy = hy - s.ry;
        std::string trail;
        for (int q = j + 1; q < k; ++q) trail += "                " + point_stmt(p.stages[q]) + "\n";
        o << "    {  // window stage " << (j - g.first) << (stencil ? ": stencil " : ": window sum ") << 2 * s.rx + 1
          << "x" << 2 * s.ry + 1 << "\n"
          << "        constexpr int RX = " << s.rx << ", RY = " << s.ry << ", OHX = " << ohx << ", OHY = " << ohy
          << ";\n        constexpr int OW = TW + 2 * OHX, OH = TH + 2 * OHY, BX = HX - OHX, BY = HY - OHY;\n"
          << "        const float* src = bufs[" << (step & 1) << "];\n"
          << "        float* dst = bufs[" << ((step + 1) & 1) << "];\n";
        if (stencil) {
            o << "        constexpr float w[" << (2 * s.rx + 1) * (2 * s.ry + 1) << "] = {";
            const int off = p.gwoff[j];
            for (int q = 0; q < (2 * s.rx + 1) * (2 * s.ry + 1); ++q)
                o << (q ? ", " : "") << flit(p.gweights[off + q]);
            o << "};\n";
        }
        // interior: GQ cells per thread, rows read once into registers
        o << "        if (interior) {\n"
             "            constexpr int NQ = (OW + GQ - 1) / GQ;\n"
             "            for (int e = threadIdx.x; e < NQ * OH; e += 256) {\n"
             "                const int cy = e / NQ, cx = (e - cy * NQ) * GQ;\n"
             "                const int lx = BX + cx, ly = BY + cy, base = ly * RW + lx;\n"
             "                float acc[GQ];\n"
             "#pragma unroll\n"
             "                for (int c = 0; c < GQ; ++c) acc[c] = 0.0f;\n"
             "#pragma unroll\n"
             "                for (int v = -RY; v <= RY; ++v) {\n"
             "                    float x[GQ + 2 * RX];\n"
             "#pragma unroll\n"
             "                    for (int q = 0; q < GQ + 2 * RX; ++q) x[q] = src[base + v * RW - RX + q];\n";
        if (stencil)
            o << "#pragma unroll\n"
                 "                    for (int u = -RX; u <= RX; ++u) {\n"
                 "                        const float wv = w[(v + RY) * (2 * RX + 1) + (u + RX)];\n"
                 "#pragma unroll\n"
                 "                        for (int c = 0; c < GQ; ++c) acc[c] = fmaf(wv, x[c + u + RX], acc[c]);\n"
                 "                    }\n";
        else
            o << "#pragma unroll\n"
                 "                    for (int c = 0; c < GQ; ++c) {\n"
                 "                        float h = 0.0f;\n"
                 "#pragma unroll\n"
                 "                        for (int u = -RX; u <= RX; ++u) h = h + x[c + u + RX];\n"
                 "                        acc[c] = acc[c] + h;\n"
                 "                    }\n";
        o << "                }\n"
             "                const int nk = OW - cx < GQ ? OW - cx : GQ;\n"
             "#pragma unroll\n"
             "                for (int c = 0; c < GQ; ++c) {\n"
             "                    if (c >= nk) break;\n"
             "                    float v = acc[c];\n"
          << trail;
        if (last)
            o << "                    out[fbase + (size_t)(oy + ly) * W + (ox + lx + c)] = v;\n";
        else
            o << "                    dst[base + c] = v;\n";
        o << "                }\n            }\n"
             "        } else {\n"
             "            for (int e = threadIdx.x; e < OW * OH; e += 256) {\n"
             "                const int cy = e / OW, cx = e - cy * OW;\n"
             "                const int lx = BX + cx, ly = BY + cy, gx = ox + lx, gy = oy + ly;\n"
             "                if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;\n"
             "                float acc = 0.0f;\n"
             "#pragma unroll\n"
             "                for (int v = -RY; v <= RY; ++v) {\n"
             "                    const int row = (clampi(gy + v, 0, H - 1) - oy) * RW - ox;\n";
        if (stencil)
            o << "#pragma unroll\n"
                 "                    for (int u = -RX; u <= RX; ++u)\n"
                 "                        acc = fmaf(w[(v + RY) * (2 * RX + 1) + (u + RX)], "
                 "src[row + clampi(gx + u, 0, W - 1)], acc);\n";
        else
            o << "                    float h = 0.0f;\n"
                 "#pragma unroll\n"
                 "                    for (int u = -RX; u <= RX; ++u) h = h + src[row + clampi(gx + u, 0, W - 1)];\n"
                 "                    acc = acc + h;\n";
        o << "                }\n"
             "                float v = acc;\n"
          << trail;
        if (last)
            o << "                out[fbase + (size_t)gy * W + gx] = v;\n";
        else
            o << "                dst[ly * RW + lx] = v;\n";
        o << "            }\n        }\n    }\n";
        if (!last) o << "    __syncthreads();\n";
        hx = ohx;
        hy = ohy;
        ++step;
        j = k;
    }
    o << "}\n";
    return o.str();
}

// One point or IIR stage on `v` (cell: the expression of its box cell, for an
// IIR's state).
static std::string trail_stmt(const fz_stage& s, const GStage& gs, const std::string& cell)
{
    if (s.op != FZ_OP_IIR) return point_stmt(s);
    const std::string a = "(double)" + flit(s.param[0]);
    return "{ double* sp = (double*)(lds + " + std::to_string(gs.buf) + ") + (" + cell +
           "); const double x = (double)v; const double y = fma(" + a + ", x, (1.0 - " + a +
           ") * (first ? x : *sp)); *sp = y; v = (float)y; }";
}

// The frame-marching kernel of a group with a temporal stage, written out
// (the same steps and arithmetic as k_gmarch, stage list as constants).
static std::string jit_march_source(const fz_plan& p, const Segment& g)
{
    std::ostringstream o;
    const int TW = g.tile_w, TH = g.tile_h, HX = g.halo, HY = g.halo_y;
    const int n = g.last - g.first + 1;
    GStage st[G_MAX_STAGES];
    g_stage_list(p.stages.data(), g.first, g.last, st);
    const int floats = march_layout(st, n, (TW + 2 * HX) * (TH + 2 * HY)) + GEN_PAD;
    const int ck_n = g.ckpt ? g_ckpt_iirs(st, n) : 0;
    const bool u8 = p.stages[g.first].in_dtype == FZ_U8;
    o << "#define GQ 5\n"
         "__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }\n"
         "extern \"C\" __global__ __launch_bounds__(256) void fz_jit(const "
      << (u8 ? "unsigned char" : "float")
      << "* __restrict__ in, float* __restrict__ out, int W, int H, int tiles_x, int tiles_y, int T, int tt, "
         "int ht, const double* __restrict__ ckpt)\n{\n"
      << "    constexpr int TW = " << TW << ", TH = " << TH << ", HX = " << HX << ", HY = " << HY
      << ", RW = TW + 2 * HX, RH = TH + 2 * HY, CELLS = RW * RH;\n"
      << "    __shared__ double lds_d[" << (floats + 1) / 2 << "];\n"
      << "    float* lds = (float*)lds_d;\n"
         "    const int nb = gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;\n"
         "    int b = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + slot;\n"
         "    const int tx = b % tiles_x;\n    b /= tiles_x;\n    const int ty = b % tiles_y;\n"
         "    const int t0 = (b / tiles_y) * tt, t1 = min(T, t0 + tt), fs = max(0, t0 - ht);\n"
         "    const int ox = tx * TW - HX, oy = ty * TH - HY;\n"
         "    const size_t P = (size_t)W * H;\n"
         "    const bool interior = ox >= 0 && oy >= 0 && ox + RW <= W && oy + RH <= H;\n";
    int lead = 0;
    while (lead < n && !g_is_window(st[lead].kind)) ++lead;
    if (ck_n > 0) {
        o << "    if (t0 > 0) {  // the leading IIRs resume from the first pass's state after frame t0 - 1\n"
             "        const double* ck = ckpt + (size_t)(t0 / tt - 1) * "
          << ck_n
          << " * P;\n"
             "        for (int e = threadIdx.x; e < CELLS; e += 256) {\n"
             "            const int ly = e / RW, lx = e - ly * RW, gx = ox + lx, gy = oy + ly;\n"
             "            if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;\n";
        int k = 0;
        for (int j = 0; j < lead; ++j)
            if (st[j].kind == G_IIR)
                o << "            ((double*)(lds + " << st[j].buf << "))[e] = ck[(size_t)" << k++
                  << " * P + (size_t)gy * W + gx];\n";
        o << "        }\n        __syncthreads();\n    }\n";
    }
    o << "    for (int f = fs; f < t1; ++f) {\n"
         "        const bool first = f == 0;\n"
         "        const size_t fbase = (size_t)f * P;\n"
         "        {\n"
         "            float* dst = lds + "
      << st[lead].buf << " + (f % " << st[lead].slots
      << ") * CELLS;\n"
         "            for (int e = threadIdx.x; e < CELLS; e += 256) {\n"
         "                const int ly = e / RW, lx = e - ly * RW, gx = ox + lx, gy = oy + ly;\n"
         "                if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;\n"
         "                float v = (float)in[fbase + (size_t)gy * W + gx];\n";
    for (int j = 0; j < lead; ++j) o << "                " << trail_stmt(p.stages[g.first + j], st[j], "e") << "\n";
    o << "                dst[e] = v;\n            }\n        }\n        __syncthreads();\n";
    int i = lead, hx = HX, hy = HY, back = 0;
    while (i < n) {
        const GStage& s = st[i];
        int j = i + 1;
        while (j < n && !g_is_window(st[j].kind)) ++j;
        const bool last = j == n;
        back += s.rt;
        const int ohx = hx - s.rx, ohy = hy - s.ry;
        const bool stencil = s.kind == G_STENCIL;
        const int nw = (2 * s.rx + 1) * (2 * s.ry + 1);
        auto trail = [&](const std::string& cell, const char* ind) {
            std::string r;
            for (int q = i + 1; q < j; ++q) r += std::string(ind) + trail_stmt(p.stages[g.first + q], st[q], cell) + "\n";
            return r;
        };
        o << "        {  // window stage " << i << "\n"
          << "            constexpr int RX = " << s.rx << ", RY = " << s.ry << ", RT = " << s.rt << ", OHX = " << ohx
          << ", OHY = " << ohy << ";\n"
          << "            constexpr int OW = TW + 2 * OHX, OH = TH + 2 * OHY, BX = HX - OHX, BY = HY - OHY;\n"
          << "            if ((fs == 0 || f >= fs + " << back << ")" << (last ? " && f >= t0" : "") << ") {\n";
        if (stencil) {
            o << "                constexpr float w[" << nw * (s.rt + 1) << "] = {";
            for (int q = 0; q < nw * (s.rt + 1); ++q) o << (q ? ", " : "") << flit(p.gweights[p.gwoff[g.first + i] + q]);
            o << "};\n";
        }
        if (!last) o << "                float* dst = lds + " << st[j].buf << " + (f % " << st[j].slots << ") * CELLS;\n";
        o << "                if (interior) {\n"
             "                    constexpr int NQ = (OW + GQ - 1) / GQ;\n"
             "                    for (int e = threadIdx.x; e < NQ * OH; e += 256) {\n"
             "                        const int cy = e / NQ, cx = (e - cy * NQ) * GQ;\n"
             "                        const int lx = BX + cx, ly = BY + cy, base = ly * RW + lx;\n"
             "                        float acc[GQ];\n"
             "#pragma unroll\n"
             "                        for (int c = 0; c < GQ; ++c) acc[c] = 0.0f;\n"
             "#pragma unroll\n"
             "                        for (int tau = 0; tau <= RT; ++tau) {\n"
             "                            const float* src = lds + "
          << s.buf << " + (max(f - tau, 0) % " << s.slots
          << ") * CELLS;\n"
             "#pragma unroll\n"
             "                            for (int v = -RY; v <= RY; ++v) {\n"
             "                                float x[GQ + 2 * RX];\n"
             "#pragma unroll\n"
             "                                for (int q = 0; q < GQ + 2 * RX; ++q) x[q] = src[base + v * RW - RX + q];\n";
        if (stencil)
            o << "#pragma unroll\n"
                 "                                for (int u = -RX; u <= RX; ++u) {\n"
                 "                                    const float wv = w[tau * " << nw << " + (v + RY) * (2 * RX + 1) + (u + RX)];\n"
                 "#pragma unroll\n"
                 "                                    for (int c = 0; c < GQ; ++c) acc[c] = fmaf(wv, x[c + u + RX], acc[c]);\n"
                 "                                }\n";
        else
            o << "#pragma unroll\n"
                 "                                for (int c = 0; c < GQ; ++c) {\n"
                 "                                    float h = 0.0f;\n"
                 "#pragma unroll\n"
                 "                                    for (int u = -RX; u <= RX; ++u) h = h + x[c + u + RX];\n"
                 "                                    acc[c] = acc[c] + h;\n"
                 "                                }\n";
        o << "                            }\n"
             "                        }\n"
             "                        const int nk = OW - cx < GQ ? OW - cx : GQ;\n"
             "#pragma unroll\n"
             "                        for (int c = 0; c < GQ; ++c) {\n"
             "                            if (c >= nk) break;\n"
             "                            float v = acc[c];\n"
          << trail("base + c", "                            ");
        if (last)
            o << "                            out[fbase + (size_t)(oy + ly) * W + (ox + lx + c)] = v;\n";
        else
            o << "                            dst[base + c] = v;\n";
        o << "                        }\n                    }\n"
             "                } else {\n"
             "                    for (int e = threadIdx.x; e < OW * OH; e += 256) {\n"
             "                        const int cy = e / OW, cx = e - cy * OW;\n"
             "                        const int lx = BX + cx, ly = BY + cy, gx = ox + lx, gy = oy + ly;\n"
             "                        if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;\n"
             "                        float acc = 0.0f;\n"
             "#pragma unroll\n"
             "                        for (int tau = 0; tau <= RT; ++tau) {\n"
             "                            const float* src = lds + "
          << s.buf << " + (max(f - tau, 0) % " << s.slots
          << ") * CELLS;\n"
             "#pragma unroll\n"
             "                            for (int v = -RY; v <= RY; ++v) {\n"
             "                                const int row = (clampi(gy + v, 0, H - 1) - oy) * RW - ox;\n";
        if (stencil)
            o << "#pragma unroll\n"
                 "                                for (int u = -RX; u <= RX; ++u)\n"
                 "                                    acc = fmaf(w[tau * " << nw << " + (v + RY) * (2 * RX + 1) + (u + RX)], "
                 "src[row + clampi(gx + u, 0, W - 1)], acc);\n";
        else
            o << "                                float h = 0.0f;\n"
                 "#pragma unroll\n"
                 "                                for (int u = -RX; u <= RX; ++u) h = h + src[row + clampi(gx + u, 0, W - 1)];\n"
                 "                                acc = acc + h;\n";
        o << "                            }\n"
             "                        }\n"
             "                        float v = acc;\n"
          << trail("ly * RW + lx", "                        ");
        if (last)
            o << "                        out[fbase + (size_t)gy * W + gx] = v;\n";
        else
            o << "                        dst[ly * RW + lx] = v;\n";
        o << "                    }\n                }\n            }\n        }\n";
        if (!last) o << "        __syncthreads();\n";
        hx = ohx;
        hy = ohy;
        i = j;
    }
    o << "        __syncthreads();\n    }\n}\n";
    return o.str();
}

namespace {
struct Compiled {
    std::vector<char> code;
};
std::mutex g_jit_mu;
std::map<std::string, Compiled> g_code;                       // source -> code object
std::map<std::pair<int, std::string>, hipFunction_t> g_func;  // (device, source) -> kernel
}  // namespace

// Compile (or find) the code object of a source; FZ_OK or FZ_E_UNSUPPORTED
// with the compiler's log.
static fz_status jit_compile_locked(const std::string& src, const Compiled** out)
{
    auto it = g_code.find(src);
    if (it != g_code.end()) {
        *out = &it->second;
        return FZ_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "fz_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(FZ_E_UNSUPPORTED, "hipRTC: cannot create the program");
    // the library's own flags: gfx950, no contraction, no packed FP32
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(FZ_E_UNSUPPORTED, "hipRTC compile failed: " + log);
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    Compiled c;
    c.code.resize(n);
    hiprtcGetCode(prog, c.code.data());
    hiprtcDestroyProgram(&prog);
    auto ins = g_code.emplace(src, std::move(c));
    *out = &ins.first->second;
    return FZ_OK;
}

fz_status jit_prepare(const fz_plan& p, const Segment& g)
{
    std::lock_guard<std::mutex> lock(g_jit_mu);
    const Compiled* c = nullptr;
    return jit_compile_locked(jit_source(p, g), &c);
}

// The kernel of group g on the current device: compiled if needed, its
// module loaded once per device (kept for the life of the process).
static hipError_t jit_function(const fz_plan& p, const Segment& g, hipFunction_t* fn)
{
    const std::string src = jit_source(p, g);
    std::lock_guard<std::mutex> lock(g_jit_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto key = std::make_pair(dev, src);
    auto it = g_func.find(key);
    if (it != g_func.end()) {
        *fn = it->second;
        return hipSuccess;
    }
    const Compiled* c = nullptr;
    if (jit_compile_locked(src, &c) != FZ_OK) return hipErrorInvalidImage;
    hipModule_t mod;
    e = hipModuleLoadData(&mod, c->code.data());
    if (e != hipSuccess) return e;
    e = hipModuleGetFunction(fn, mod, "fz_jit");
    if (e != hipSuccess) return e;
    g_func.emplace(key, *fn);
    return hipSuccess;
}

int jit_load(const fz_plan& p, const Segment& g)
{
    hipFunction_t fn = nullptr;
    return (int)jit_function(p, g, &fn);
}

int launch_jit(const fz_plan& p, const Segment& g, const void* in, void* out, const void* ckpt, void* stream)
{
    hipFunction_t fn = nullptr;
    const hipError_t e = jit_function(p, g, &fn);
    if (e != hipSuccess) return (int)e;
    GStage st[G_MAX_STAGES];
    g_stage_list(p.stages.data(), g.first, g.last, st);
    int ht = 0;
    if (g_temporal(st, g.last - g.first + 1, nullptr, &ht)) {  // the frame-marching form
        const int tiles_x = (p.W + g.tile_w - 1) / g.tile_w, tiles_y = (p.H + g.tile_h - 1) / g.tile_h;
        const long long blocks = (long long)tiles_x * tiles_y * ((p.T + g.tpb - 1) / g.tpb);
        if (blocks > 0x7fffffffLL || g.tpb < 1) return (int)hipErrorInvalidConfiguration;
        int W = p.W, H = p.H, txs = tiles_x, tys = tiles_y, T = p.T, tt = g.tpb, hts = ht;
        const void* pin = in;
        float* pout = (float*)out;
        const void* pck = ckpt;
        void* args[] = {&pin, &pout, &W, &H, &txs, &tys, &T, &tt, &hts, &pck};
        return (int)hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, BLOCK_THREADS, 1, 1, 0, (hipStream_t)stream,
                                          args, nullptr);
    }
    const int tiles_x = (p.W + g.tile_w - 1) / g.tile_w, tiles_y = (p.H + g.tile_h - 1) / g.tile_h;
    const long long blocks = (long long)tiles_x * tiles_y * p.T;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    int W = p.W, H = p.H, txs = tiles_x, tys = tiles_y;
    const void* pin = in;
    float* pout = (float*)out;
    void* args[] = {&pin, &pout, &W, &H, &txs, &tys};
    return (int)hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, BLOCK_THREADS, 1, 1, 0, (hipStream_t)stream, args,
                                      nullptr);
}

}  // namespace fz
