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
// one straight to global memory) and each output's arithmetic in the same
// order, so its output equals the tile kernel's in value (the sign of a zero
// sum aside); the work per thread differs: a block of neighbouring cells
// (five across, up to two down) per thread, and aligned four-cell loads of
// the input box.  Groups with a temporal stage get the frame-marching kernel
// written out the same way (rings of earlier frames per stencil, IIR states,
// checkpoint restore).
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
#include "jit_layout.h"

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

// The group's kernel.  One form serves every generic window group: a work
// item is an output tile and a run of tt frames (tt = 1 and no temporal halo
// for a group without temporal stages).  Borders: a tile whose box leaves the
// frame loads its out-of-frame cells with clamped reads (the replicate border
// of the group's input) and, after every window stage but the last, copies
// each out-of-frame cell of that stage's output from the frame cell it
// clamps to (the replicate border of that stage's output); so every stage
// runs the unclamped path everywhere, and its in-frame results are exactly
// those of clamped reads.  The last stage stores its in-frame cells only.
// The input box of a tile that lies inside the frame across (every tile but
// the left and right border ones) is read four cells per load, aligned, with
// its rows clamped; others cell by cell with both coordinates clamped.
std::string jit_source(const fz_plan& p, const Segment& g)
{
    std::ostringstream o;
    const int TW = g.tile_w, TH = g.tile_h, HX = g.halo, HY = g.halo_y;
    const int n = g.last - g.first + 1;
    GStage st[G_MAX_STAGES];
    g_stage_list(p.stages.data(), g.first, g.last, st);
    const int LP = jit_pitch(st, n, TW, TH, HX, HY);
    const int floats = jit_layout(st, n, LP * (TH + 2 * HY)) + GEN_PAD;
    const int ck_n = g.ckpt ? g_ckpt_iirs(st, n) : 0;
    const bool u8 = p.stages[g.first].in_dtype == FZ_U8;
    const int S = (4 - HX % 4) % 4;  // tiles are a multiple of 4 wide: ox = tx TW - HX = S (mod 4)
    o << "__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }\n"
         "extern \"C\" __global__ __launch_bounds__(256) void fz_jit(const "
      << (u8 ? "unsigned char" : "float")
      << "* __restrict__ in, float* __restrict__ out, int W, int H, int tiles_x, int tiles_y, int T, int tt, "
         "int ht, const double* __restrict__ ckpt)\n{\n"
      << "    constexpr int TW = " << TW << ", TH = " << TH << ", HX = " << HX << ", HY = " << HY
      << ", RW = TW + 2 * HX, RH = TH + 2 * HY, LP = " << LP
      << ", CELLS = LP * RH, BOX = RW * RH;  // LP: LDS row pitch\n"
      << "    constexpr int S = " << S << ", ND = (RW + S + 3) / 4, NV = RH * ND;  // four-cell groups of the box\n"
      << "    __shared__ double lds_d[" << (floats + 1) / 2 << "];\n"
      << "    float* lds = (float*)lds_d;\n"
         // blocks dealt to XCDs round-robin: contiguous runs of tiles per XCD
         "    const int nb = gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;\n"
         "    int b = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + slot;\n"
         "    const int tx = b % tiles_x;\n    b /= tiles_x;\n    const int ty = b % tiles_y;\n"
         "    const int t0 = (b / tiles_y) * tt, t1 = min(T, t0 + tt), fs = max(0, t0 - ht);\n"
         "    const int ox = tx * TW - HX, oy = ty * TH - HY;\n"
         "    const size_t P = (size_t)W * H;\n"
         "    const bool interior = ox >= 0 && oy >= 0 && ox + RW <= W && oy + RH <= H;\n"
         "    const bool xin = ox >= 0 && ox + RW <= W && (W & 3) == 0 && ((size_t)in & "
      << (u8 ? 3 : 15)
      << ") == 0;\n"
         "    const bool vec_out = interior && (W & 3) == 0 && ((size_t)out & 15) == 0;\n";
    int lead = 0;
    while (lead < n && !g_is_window(st[lead].kind)) ++lead;
    // The input box is handled in four-cell groups (row ly, group kd: cells
    // lx = 4 kd + q - S, q = 0..3), group it = ly ND + kd by thread it mod
    // 256, the same threads every frame: groups of a tile inside the frame
    // across are loaded with one aligned load, others cell by cell with
    // clamped coordinates.  A leading IIR's double states are the thread's
    // registers ist<j>[k][q] (k: its k-th group), restored from the
    // checkpoint of the run before.
    o << "    constexpr int NLV = (NV + 255) / 256, NPF = " << (u8 ? "NLV" : "4 * NLV") << ";\n"
         "    const int a0 = ox - S;\n"
         "    unsigned int pf[NPF];  // the next box: four u8 cells or one f32 cell per word\n";
    int n_lead_iir = 0;
    for (int j = 0; j < lead; ++j)
        if (st[j].kind == G_IIR) o << "    double ist" << n_lead_iir++ << "[NLV][4];\n";
    if (ck_n > 0) {
        o << "    if (t0 > 0) {  // the leading IIRs resume from the first pass's state after frame t0 - 1\n"
             "        const double* ck = ckpt + (size_t)(t0 / tt - 1) * "
          << ck_n
          << " * P;\n"
             "#pragma unroll\n"
             "        for (int k = 0; k < NLV; ++k) {\n"
             "            const int it = threadIdx.x + 256 * k;\n"
             "            if (it < NV) {\n"
             "                const int ly = it / ND, kd = it - ly * ND;\n"
             "#pragma unroll\n"
             "                for (int q = 0; q < 4; ++q) {\n"
             "                    const int lx = 4 * kd + q - S;\n"
             "                    if (lx < 0 || lx >= RW) continue;\n"
             "                    const size_t gi = (size_t)clampi(oy + ly, 0, H - 1) * W + clampi(ox + lx, 0, W - 1);\n";
        for (int k = 0; k < n_lead_iir; ++k) o << "                    ist" << k << "[k][q] = ck[(size_t)" << k << " * P + gi];\n";
        o << "                }\n            }\n        }\n    }\n";
    }
    std::string lead_stmts;
    {
        int k = 0;
        for (int j = 0; j < lead; ++j) {
            const fz_stage& fs = p.stages[g.first + j];
            if (st[j].kind == G_IIR) {
                const std::string a = "(double)" + flit(fs.param[0]), r = "ist" + std::to_string(k++) + "[k][Q]";
                lead_stmts += "                        { const double x = (double)v; const double y = fma(" + a + ", x, (1.0 - " +
                              a + ") * (first ? x : " + r + ")); " + r + " = y; v = (float)y; }\n";
            } else {
                lead_stmts += "                        " + point_stmt(fs) + "\n";
            }
        }
    }
    const char* vt = u8 ? "unsigned int" : "float4";
    auto issue = [&](const std::string& frame) {
        std::ostringstream q;
        q << "        {  // loads of frame " << frame << "'s box\n"
          << "            const size_t gb = (size_t)(" << frame << ") * P;\n"
             "#pragma unroll\n"
             "            for (int k = 0; k < NLV; ++k) {\n"
             "                const int it = threadIdx.x + 256 * k;\n"
             "                if (it < NV) {\n"
             "                    const int ly = it / ND, kd = it - ly * ND;\n"
             "                    const size_t rb = gb + (size_t)clampi(oy + ly, 0, H - 1) * W;\n"
             "                    if (xin) {\n"
             "                        const "
          << vt << " w = *(const " << vt << "*)(in + rb + a0 + 4 * kd);\n";
        if (u8)
            q << "                        pf[k] = w;\n";
        else
            q << "                        pf[4 * k] = __float_as_uint(w.x);\n"
                 "                        pf[4 * k + 1] = __float_as_uint(w.y);\n"
                 "                        pf[4 * k + 2] = __float_as_uint(w.z);\n"
                 "                        pf[4 * k + 3] = __float_as_uint(w.w);\n";
        q << "                    } else {\n";
        if (u8)
            q << "                        unsigned int w = 0;\n";
        q << "#pragma unroll\n"
             "                        for (int q = 0; q < 4; ++q) {\n"
             "                            const int lx = 4 * kd + q - S;\n"
             "                            if (lx < 0 || lx >= RW) continue;\n";
        if (u8)
            q << "                            w |= (unsigned int)in[rb + clampi(ox + lx, 0, W - 1)] << (8 * q);\n";
        else
            q << "                            pf[4 * k + q] = __float_as_uint(in[rb + clampi(ox + lx, 0, W - 1)]);\n";
        q << "                        }\n";
        if (u8) q << "                        pf[k] = w;\n";
        q << "                    }\n"
             "                }\n"
             "            }\n"
             "        }\n";
        return q.str();
    };
    const char* vx[4] = {"(float)(pf[k] & 255u)", "(float)((pf[k] >> 8) & 255u)", "(float)((pf[k] >> 16) & 255u)",
                         "(float)(pf[k] >> 24)"};
    o << "    if (fs < t1)\n"
      << issue("fs")
      << "    for (int f = fs; f < t1; ++f) {\n"
         "        const bool first = f == 0;\n"
         "        const size_t fbase = (size_t)f * P;\n"
         "        float* dst = lds + "
      << st[lead].buf << " + (f % " << st[lead].slots << ") * CELLS;\n"
      << "#pragma unroll\n"
         "        for (int k = 0; k < NLV; ++k) {\n"
         "            const int it = threadIdx.x + 256 * k;\n"
         "            if (it < NV) {\n"
         "                const int ly = it / ND, kd = it - ly * ND;\n";
    for (int q = 0; q < 4; ++q) {
        std::string ls = lead_stmts;
        for (size_t pos; (pos = ls.find("[k][Q]")) != std::string::npos;) ls.replace(pos, 6, "[k][" + std::to_string(q) + "]");
        o << "                if (" << (q < S ? "kd > 0 && " : "") << "4 * kd + " << q - S << " < RW) {\n"
          << "                    float v = " << (u8 ? std::string(vx[q]) : "__uint_as_float(pf[4 * k + " + std::to_string(q) + "])")
          << ";\n"
          << ls << "                    dst[ly * LP + 4 * kd + " << q - S << "] = v;\n                }\n";
    }
    o << "            }\n"
         "        }\n"
         "        __syncthreads();\n"
         "        if (f + 1 < t1)\n"
      << issue("f + 1");
    int back = 0;
    for (const WinStep& ws : win_steps(st, n, TW, TH, HX, HY)) {
        const int i = ws.i, j = ws.j, ohx = ws.ohx, ohy = ws.ohy, gq = ws.gq, gr = ws.gr;
        const bool last = ws.last;
        const GStage& s = st[i];
        back += s.rt;
        const bool stencil = s.kind == G_STENCIL;
        const int nw = (2 * s.rx + 1) * (2 * s.ry + 1);
        std::string trail;
        for (int q = i + 1; q < j; ++q)
            trail += "                            " + trail_stmt(p.stages[g.first + q], st[q], "base + r * LP + c") + "\n";
        o << "        {  // window stage " << i << (stencil ? ": stencil " : ": window sum ") << 2 * s.rx + 1 << "x"
          << 2 * s.ry + 1 << (s.rt ? " over " + std::to_string(s.rt + 1) + " frames" : std::string()) << "\n"
          << "            constexpr int RX = " << s.rx << ", RY = " << s.ry << ", RT = " << s.rt << ", OHX = " << ohx
          << ", OHY = " << ohy << ", GR = " << gr << ", GQ = " << gq << ";\n"
          << "            constexpr int OW = TW + 2 * OHX, OH = TH + 2 * OHY, BX = HX - OHX, BY = HY - OHY;\n";
        if (!last) o << "            float* dst = lds + " << st[j].buf << " + (f % " << st[j].slots << ") * CELLS;\n";
        o << "            if ((fs == 0 || f >= fs + " << back << ")" << (last ? " && f >= t0" : "") << ") {\n";
        if (stencil) {
            o << "                constexpr float w[" << nw * (s.rt + 1) << "] = {";
            for (int q = 0; q < nw * (s.rt + 1); ++q) o << (q ? ", " : "") << flit(p.gweights[p.gwoff[g.first + i] + q]);
            o << "};\n";
        }
        // a block of GQ x GR cells per thread; the last row block is moved up
        // to end at the region's last row (no reads past the buffer) and skips
        // the rows the block above it owns
        o << "                constexpr int NQ = (OW + GQ - 1) / GQ, NR = (OH + GR - 1) / GR;\n"
             "                for (int e = threadIdx.x; e < NQ * NR; e += 256) {\n"
             "                    const int ry = e / NQ, cx = (e - ry * NQ) * GQ;\n"
             "                    const int cy = min(ry * GR, OH - GR), skip = ry * GR - cy;\n"
             "                    const int lx = BX + cx, ly = BY + cy, base = ly * LP + lx;\n"
             "                    float acc[GR][GQ];\n"
             "#pragma unroll\n"
             "                    for (int r = 0; r < GR; ++r)\n"
             "#pragma unroll\n"
             "                        for (int c = 0; c < GQ; ++c) acc[r][c] = "
          << (stencil ? "0.0f" : "-0.0f")
          << ";\n"
             "#pragma unroll\n"
             "                    for (int tau = 0; tau <= RT; ++tau) {\n"
             "                        const float* src = lds + "
          << s.buf << " + (max(f - tau, 0) % " << s.slots
          << ") * CELLS;\n"
             "#pragma unroll\n"
             "                        for (int v = -RY; v < GR + RY; ++v) {\n"
             "                            float x[GQ + 2 * RX];\n"
             "#pragma unroll\n"
             "                            for (int q = 0; q < GQ + 2 * RX; ++q) x[q] = src[base + v * LP - RX + q];\n";
        if (stencil)
            o << "#pragma unroll\n"
                 "                            for (int r = 0; r < GR; ++r) {\n"
                 "                                if (v - r < -RY || v - r > RY) continue;\n"
                 "#pragma unroll\n"
                 "                                for (int u = -RX; u <= RX; ++u) {\n"
                 "                                    const float wv = w[tau * " << nw << " + (v - r + RY) * (2 * RX + 1) + (u + RX)];\n"
                 "#pragma unroll\n"
                 "                                    for (int c = 0; c < GQ; ++c) acc[r][c] = fmaf(wv, x[c + u + RX], acc[r][c]);\n"
                 "                                }\n"
                 "                            }\n";
        else
            o << "                            float h[GQ];\n"
                 "#pragma unroll\n"
                 "                            for (int c = 0; c < GQ; ++c) {\n"
                 "                                h[c] = x[c];\n"
                 "#pragma unroll\n"
                 "                                for (int u = 1; u <= 2 * RX; ++u) h[c] = h[c] + x[c + u];\n"
                 "                            }\n"
                 "#pragma unroll\n"
                 "                            for (int r = 0; r < GR; ++r) {\n"
                 "                                if (v - r < -RY || v - r > RY) continue;\n"
                 "#pragma unroll\n"
                 "                                for (int c = 0; c < GQ; ++c) acc[r][c] = acc[r][c] + h[c];\n"
                 "                            }\n";
        o << "                        }\n"
             "                    }\n"
             "                    const int nk = OW - cx < GQ ? OW - cx : GQ;\n"
             "#pragma unroll\n"
             "                    for (int r = 0; r < GR; ++r) {\n"
             "                        if (r < skip) continue;\n";
        if (last)
            o << "                        const int gy = oy + ly + r, gx0 = ox + lx;\n"
                 "                        const bool row_in = gy >= 0 && gy < H;\n"
                 "                        float* orow = out + fbase + (size_t)gy * W + gx0;\n";
        if (last)
            o << "                        if (vec_out) {  // a tile inside the frame: GQ = 4 cells, 16-byte aligned\n"
                 "                            float vv[GQ];\n"
                 "#pragma unroll\n"
                 "                            for (int c = 0; c < GQ; ++c) {\n"
                 "                                float v = acc[r][c];\n"
              << trail
              << "                                vv[c] = v;\n"
                 "                            }\n"
                 "                            *(float4*)orow = make_float4(vv[0], vv[1], vv[2], vv[3]);\n"
                 "                            continue;\n"
                 "                        }\n";
        o << "#pragma unroll\n"
             "                        for (int c = 0; c < GQ; ++c) {\n"
             "                            if (c >= nk) break;\n"
             "                            float v = acc[r][c];\n"
          << trail;
        if (last)
            o << "                            if (interior || (row_in && gx0 + c >= 0 && gx0 + c < W)) orow[c] = v;\n";
        else
            o << "                            dst[base + r * LP + c] = v;\n";
        o << "                        }\n                    }\n                }\n            }\n";
        if (!last) {
            // replicate border of this stage's output for the next stage: only
            // the out-of-frame cells are visited -- whole rows above and below
            // the frame, then the columns left and right of it on frame rows
            o << "            __syncthreads();\n"
                 "            if (!interior) {\n"
                 "                const int y0 = clampi(-oy - BY, 0, OH), y1 = clampi(H - oy - BY, y0, OH);\n"
                 "                const int x0 = clampi(-ox - BX, 0, OW), x1 = clampi(W - ox - BX, x0, OW);\n"
                 "                const int na = (OH - (y1 - y0)) * OW, ncol = x0 + OW - x1, nall = na + (y1 - y0) * ncol;\n"
                 "                for (int e = threadIdx.x; e < nall; e += 256) {\n"
                 "                    int cy, cx;\n"
                 "                    if (e < na) {\n"
                 "                        const int r = e / OW;\n"
                 "                        cx = e - r * OW;\n"
                 "                        cy = r < y0 ? r : r - y0 + y1;\n"
                 "                    } else {\n"
                 "                        const int r = (e - na) / ncol, k = e - na - r * ncol;\n"
                 "                        cy = y0 + r;\n"
                 "                        cx = k < x0 ? k : k - x0 + x1;\n"
                 "                    }\n"
                 "                    const int lx = BX + cx, ly = BY + cy;\n"
                 "                    dst[ly * LP + lx] = dst[(clampi(oy + ly, 0, H - 1) - oy) * LP + (clampi(ox + lx, 0, W - 1) - ox)];\n"
                 "                }\n"
                 "                __syncthreads();\n"
                 "            }\n";
        }
        o << "        }\n";
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
    (void)g_temporal(st, g.last - g.first + 1, nullptr, &ht);
    const int tt = g.tpb;  // frames per work item (temporal or not)
    if (tt < 1) return (int)hipErrorInvalidConfiguration;
    const int tiles_x = (p.W + g.tile_w - 1) / g.tile_w, tiles_y = (p.H + g.tile_h - 1) / g.tile_h;
    const long long blocks = (long long)tiles_x * tiles_y * ((p.T + tt - 1) / tt);
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    int W = p.W, H = p.H, txs = tiles_x, tys = tiles_y, T = p.T, tts = tt, hts = ht;
    const void* pin = in;
    float* pout = (float*)out;
    const void* pck = ckpt;
    void* args[] = {&pin, &pout, &W, &H, &txs, &tys, &T, &tts, &hts, &pck};
    return (int)hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, BLOCK_THREADS, 1, 1, 0, (hipStream_t)stream, args,
                                      nullptr);
}

}  // namespace fz
