// Fused-group kernels for gfx950.
//
// One workgroup produces an output box of TW x TH pixels over a run of frames
// (Sec. V, Fig. 3).  For a group of stages A..B (Algorithm 1):
//   1. the input box, grown by the group's halo on every side (Sec. VI-C), is
//      read once from global memory into LDS, with the group's leading point
//      stages applied in registers on the way in;
//   2. each window stage reads its neighbourhood from LDS and writes its output
//      region, grown by the halo the later stages still need, back to LDS; the
//      point stages that follow it run in registers before that write, so only
//      window stages need a barrier (thread-to-multi-thread dependence);
//   3. the last window stage's values, after the trailing point stages, go to
//      global memory.
// Frame borders are replicated per stage: a window stage computes every cell of
// its region at the nearest in-frame position, so the cells outside the frame
// hold copies of the edge values of that stage's output, which is what the
// next stage reads as its replicated input.
// Window stages that separate (Gaussian, box sums, 3x3 maximum) run as a
// horizontal pass over the input rows followed by a vertical pass.
// A group ending in the frame difference marches through its frames in order
// and keeps the previous frame's value of every output pixel in registers; it
// first computes the frame before its first one (one frame of temporal halo).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "fz_ops.h"
#include "stage_math.h"

namespace fz {

struct SegParams {
    const void* in;
    void* out;
    int W, H, T;
    int tpb;  // frames per workgroup
    Gauss5W gw;
    float k, thr;
    fz_point* points;
    uint32_t* count;
    uint32_t cap;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Last index e >= s-1 such that stages s..e are point stages other than the
// frame difference (they run in registers right after the producing step).
FZ_HD constexpr int pw_end(int ch, int s, int B)
{
    int e = s - 1;
    for (int j = s; j <= B; ++j) {
        int op = chain_op(ch, j);
        if (op_info(op).r > 0 || op == FZ_OP_FRAMEDIFF) break;
        e = j;
    }
    return e;
}
FZ_HD constexpr int next_window(int ch, int s, int B)
{
    for (int j = s; j <= B; ++j)
        if (is_window(ch, j)) return j;
    return B + 1;
}
FZ_HD constexpr bool separable(int op) { return op == FZ_OP_GAUSS5 || op == FZ_OP_BOXSUM5 || op == FZ_OP_NMS3; }

// ---------------------------------------------------------------- pixel I/O
// Read pixel (t, y, x) of the group input into v[] as floats.
template <int CH, int A>
__device__ __forceinline__ void load_px(const SegParams& p, int t, int y, int x, float* v)
{
    constexpr OpInfo o = op_info(chain_op(CH, A));
    const size_t plane = (size_t)p.W * p.H;
    const size_t off = (size_t)t * plane + (size_t)y * p.W + x;
    if constexpr (o.op == FZ_OP_RGB2GRAY) {
        const uint8_t* s = (const uint8_t*)p.in + 3 * off;
        v[0] = (float)s[0];
        v[1] = (float)s[1];
        v[2] = (float)s[2];
    } else if constexpr (o.in_dt == FZ_U8) {
        v[0] = (float)((const uint8_t*)p.in)[off];
    } else {
        const size_t vol = plane * p.T;
#pragma unroll
        for (int c = 0; c < o.in_ch; ++c) v[c] = ((const float*)p.in)[c * vol + off];
    }
}

template <int CH, int B>
__device__ __forceinline__ void store_px(const SegParams& p, int t, int y, int x, const float* v)
{
    constexpr OpInfo o = op_info(chain_op(CH, B));
    const size_t plane = (size_t)p.W * p.H;
    const size_t off = (size_t)t * plane + (size_t)y * p.W + x;
    if constexpr (o.out_dt == FZ_U8) {
        ((uint8_t*)p.out)[off] = (uint8_t)(uint32_t)v[0];
    } else {
        const size_t vol = plane * p.T;
#pragma unroll
        for (int c = 0; c < o.out_ch; ++c) ((float*)p.out)[c * vol + off] = v[c];
    }
}

// ---------------------------------------------------------------- point stages
template <int OP>
__device__ __forceinline__ void point_op(float* v, const SegParams& p)
{
    if constexpr (OP == FZ_OP_RGB2GRAY) {
        v[0] = (float)rgb2gray((uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2]);
    } else if constexpr (OP == FZ_OP_GRADMAG) {
        v[0] = gradmag(v[0], v[1]);
    } else if constexpr (OP == FZ_OP_PRODUCTS) {
        float a = v[0], b = v[1];
        products(a, b, v[0], v[1], v[2]);
    } else if constexpr (OP == FZ_OP_HARRIS) {
        v[0] = harris(v[0], v[1], v[2], p.k);
    } else if constexpr (OP == FZ_OP_THRESHOLD) {
        v[0] = threshold(v[0], p.thr);
    }
}

template <int CH, int S, int E>
__device__ __forceinline__ void point_run(float* v, const SegParams& p)
{
    if constexpr (S <= E) {
        point_op<chain_op(CH, S)>(v, p);
        point_run<CH, S + 1, E>(v, p);
    }
}

// ---------------------------------------------------------------- feature points
// Append a point per lane with `is_pt`; one atomic per wavefront.  Must be
// reached by every lane of the wavefront.
__device__ __forceinline__ void emit_points(const SegParams& p, bool is_pt, uint32_t t, uint32_t y, uint32_t x,
                                            float r)
{
    const unsigned long long m = __ballot(is_pt);
    if (m == 0ull) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(p.count, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (is_pt) {
        const uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (idx < p.cap) {
            fz_point q;
            q.t = t;
            q.y = y;
            q.x = x;
            q.response = r;
            p.points[idx] = q;
        }
    }
}

// Per-thread state of the final output cells (temporal groups).
template <int PER>
struct FinalState {
    float prev[PER];
};

// Handle one final output cell: trailing frame difference, store, points.
template <int CH, int B, bool TEMPORAL, int PER>
__device__ __forceinline__ void finish_cell(const SegParams& p, FinalState<PER>& st, int k, float* v, int t, bool real,
                                            int gy, int gx, bool inside)
{
    if constexpr (TEMPORAL) {
        if (t == 0) st.prev[k] = v[0];
        const float d = (float)framediff((uint32_t)v[0], (uint32_t)st.prev[k]);
        st.prev[k] = v[0];
        v[0] = d;
    }
    if (real && inside) store_px<CH, B>(p, t, gy, gx, v);
}

// ---------------------------------------------------------------- steps
// Load the group's input box (halo H) for frame t into buf (channel planes).
template <int CH, int A, int B, int TW, int TH, bool EDGE>
__device__ __forceinline__ void load_step(const SegParams& p, float* buf, int t, int ox0, int oy0)
{
    constexpr int H = group_halo(CH, A, B);
    constexpr int RW = TW + 2 * H, RH = TH + 2 * H, N = RW * RH;
    constexpr int CL = channels_after_load(CH, A, B);
    constexpr int E = pw_end(CH, A, B);
    for (int i = threadIdx.x; i < N; i += BLOCK_THREADS) {
        const int ry = i / RW, rx = i - ry * RW;
        int gy = oy0 - H + ry, gx = ox0 - H + rx;
        if (EDGE) {
            gy = clampi(gy, 0, p.H - 1);
            gx = clampi(gx, 0, p.W - 1);
        }
        float v[3];
        load_px<CH, A>(p, t, gy, gx, v);
        point_run<CH, A, E>(v, p);
#pragma unroll
        for (int c = 0; c < CL; ++c) buf[c * N + i] = v[c];
    }
}

// One window stage S.  `bin` holds its input region (halo hin), `bother` is
// free.  Returns nothing; the output lands in bin (separable stages: written by
// the vertical pass after the horizontal pass has consumed bin) or in bother
// (direct stages); the final window stage writes global memory instead.
template <int CH, int S, int B, int TW, int TH, bool EDGE, bool TEMPORAL, int PER>
__device__ __forceinline__ void window_step(const SegParams& p, float* bin, float* bother, int t, bool real, int ox0,
                                            int oy0, FinalState<PER>& st)
{
    constexpr int OP = chain_op(CH, S);
    constexpr OpInfo o = op_info(OP);
    constexpr int R = o.r;
    constexpr int hin = halo_after(CH, S - 1, B), hout = halo_after(CH, S, B);
    constexpr int RWi = TW + 2 * hin, RHi = TH + 2 * hin, Ni = RWi * RHi;
    constexpr int RWo = TW + 2 * hout, RHo = TH + 2 * hout, No = RWo * RHo;
    constexpr int E = pw_end(CH, S + 1, B);
    constexpr int COUT = channels_after_step(CH, S, B);
    constexpr bool FINAL = hout == 0;
    static_assert(OP != FZ_OP_NMS3 || FINAL, "suppression must be the last window stage of its group");
    static_assert(!FINAL || (TW * TH) % BLOCK_THREADS == 0, "tile must be a multiple of the block");

    if constexpr (separable(OP)) {
        constexpr int CIN = o.in_ch;
        constexpr int NT = RHi * RWo;  // horizontal-pass intermediate: input rows x output columns
        float* tmp = bother;
        // horizontal pass
        for (int i = threadIdx.x; i < NT; i += BLOCK_THREADS) {
            const int ry = i / RWo, rx = i - ry * RWo;
            int gx = ox0 - hout + rx;
            if (EDGE) gx = clampi(gx, 0, p.W - 1);
            const int lx = gx - (ox0 - hin);
            const float* row = bin + ry * RWi + lx;
#pragma unroll
            for (int c = 0; c < CIN; ++c) {
                const float* q = row + c * Ni;
                float r;
                if constexpr (OP == FZ_OP_GAUSS5)
                    r = gauss5_taps(p.gw, q[-2], q[-1], q[0], q[1], q[2]);
                else if constexpr (OP == FZ_OP_BOXSUM5)
                    r = sum5(q[-2], q[-1], q[0], q[1], q[2]);
                else
                    r = max3(q[-1], q[0], q[1]);
                tmp[c * NT + i] = r;
            }
        }
        __syncthreads();
        // vertical pass
        auto vert = [&](int ry, int rx, float* v, int& cy, int& cx) {
            int gy = oy0 - hout + ry, gx = ox0 - hout + rx;
            cy = gy;
            cx = gx;
            if (EDGE) {
                cy = clampi(gy, 0, p.H - 1);
                cx = clampi(gx, 0, p.W - 1);
            }
            const int ly = cy - (oy0 - hin);
            const float* col = tmp + ly * RWo + rx;
#pragma unroll
            for (int c = 0; c < CIN; ++c) {
                const float* q = col + c * NT;
                if constexpr (OP == FZ_OP_GAUSS5)
                    v[c] = gauss5_taps(p.gw, q[-2 * RWo], q[-RWo], q[0], q[RWo], q[2 * RWo]);
                else if constexpr (OP == FZ_OP_BOXSUM5)
                    v[c] = sum5(q[-2 * RWo], q[-RWo], q[0], q[RWo], q[2 * RWo]);
                else {
                    const float wmax = max3(q[-RWo], q[0], q[RWo]);
                    const float centre = bin[ly * RWi + (cx - (ox0 - hin))];
                    v[1] = centre;
                    v[0] = (float)nms_keep(centre, wmax);
                }
            }
        };
        if constexpr (!FINAL) {
            for (int i = threadIdx.x; i < No; i += BLOCK_THREADS) {
                const int ry = i / RWo, rx = i - ry * RWo;
                float v[3];
                int cy, cx;
                vert(ry, rx, v, cy, cx);
                point_run<CH, S + 1, E>(v, p);
#pragma unroll
                for (int c = 0; c < COUT; ++c) bin[c * No + i] = v[c];
            }
        } else {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = threadIdx.x + k * BLOCK_THREADS;
                const int ry = i / TW, rx = i - ry * TW;
                float v[3];
                int cy, cx;
                vert(ry, rx, v, cy, cx);
                const int gy = oy0 + ry, gx = ox0 + rx;
                const bool inside = gy < p.H && gx < p.W;
                if constexpr (OP == FZ_OP_NMS3) {
                    const bool is_pt = real && inside && v[0] != 0.0f && p.count != nullptr;
                    emit_points(p, is_pt, (uint32_t)t, (uint32_t)gy, (uint32_t)gx, v[1]);
                }
                point_run<CH, S + 1, E>(v, p);
                finish_cell<CH, B, TEMPORAL, PER>(p, st, k, v, t, real, gy, gx, inside);
            }
        }
    } else {
        static_assert(OP == FZ_OP_SOBEL3, "direct window stage");
        auto one = [&](int ry, int rx, float* v) {
            int gy = oy0 - hout + ry, gx = ox0 - hout + rx;
            if (EDGE) {
                gy = clampi(gy, 0, p.H - 1);
                gx = clampi(gx, 0, p.W - 1);
            }
            const int ly = gy - (oy0 - hin), lx = gx - (ox0 - hin);
            const float* q = bin + ly * RWi + lx;
            float g[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) g[a][b] = q[(a - 1) * RWi + (b - 1)];
            sobel3(g, v[0], v[1]);
        };
        if constexpr (!FINAL) {
            for (int i = threadIdx.x; i < No; i += BLOCK_THREADS) {
                const int ry = i / RWo, rx = i - ry * RWo;
                float v[3];
                one(ry, rx, v);
                point_run<CH, S + 1, E>(v, p);
#pragma unroll
                for (int c = 0; c < COUT; ++c) bother[c * No + i] = v[c];
            }
        } else {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int i = threadIdx.x + k * BLOCK_THREADS;
                const int ry = i / TW, rx = i - ry * TW;
                float v[3];
                one(ry, rx, v);
                const int gy = oy0 + ry, gx = ox0 + rx;
                point_run<CH, S + 1, E>(v, p);
                finish_cell<CH, B, TEMPORAL, PER>(p, st, k, v, t, real, gy, gx, gy < p.H && gx < p.W);
            }
        }
    }
    (void)R;
}

// Run window stages S.. of the group; CUR is the buffer holding S's input.
template <int CH, int S, int B, int TW, int TH, bool EDGE, bool TEMPORAL, int PER, int CUR>
__device__ __forceinline__ void window_chain(const SegParams& p, float* lds, int nb, int t, bool real, int ox0, int oy0,
                                             FinalState<PER>& st)
{
    if constexpr (S <= B) {
        float* bin = lds + CUR * nb;
        float* bother = lds + (1 - CUR) * nb;
        window_step<CH, S, B, TW, TH, EDGE, TEMPORAL, PER>(p, bin, bother, t, real, ox0, oy0, st);
        __syncthreads();
        constexpr int NXT = next_window(CH, S + 1, B);
        constexpr int NCUR = separable(chain_op(CH, S)) ? CUR : 1 - CUR;
        window_chain<CH, NXT, B, TW, TH, EDGE, TEMPORAL, PER, NCUR>(p, lds, nb, t, real, ox0, oy0, st);
    }
}

template <int CH, int A, int B, int TW, int TH, bool EDGE>
__device__ __forceinline__ void group_body(const SegParams& p, float* lds, int ox0, int oy0)
{
    constexpr bool TEMPORAL = chain_op(CH, B) == FZ_OP_FRAMEDIFF;
    constexpr int PER = TW * TH / BLOCK_THREADS;
    constexpr int NB = engine_buffer_floats(CH, A, B, TW, TH);
    FinalState<PER> st;
#pragma unroll
    for (int k = 0; k < PER; ++k) st.prev[k] = 0.0f;
    const int t0 = blockIdx.z * p.tpb;
    const int t1 = min(t0 + p.tpb, p.T);
    const int ts = TEMPORAL ? max(t0 - 1, 0) : t0;
    for (int t = ts; t < t1; ++t) {
        const bool real = t >= t0;
        load_step<CH, A, B, TW, TH, EDGE>(p, lds, t, ox0, oy0);
        __syncthreads();
        window_chain<CH, next_window(CH, A, B), B, TW, TH, EDGE, TEMPORAL, PER, 0>(p, lds, NB, t, real, ox0, oy0, st);
    }
}

template <int CH, int A, int B, int TW, int TH>
__global__ __launch_bounds__(BLOCK_THREADS) void k_group(SegParams p)
{
    constexpr int NB = engine_buffer_floats(CH, A, B, TW, TH);
    __shared__ float lds[2 * NB];
    constexpr int H = group_halo(CH, A, B);
    const int ox0 = blockIdx.x * TW, oy0 = blockIdx.y * TH;
    const bool edge = ox0 - H < 0 || oy0 - H < 0 || ox0 + TW + H > p.W || oy0 + TH + H > p.H;
    if (edge)
        group_body<CH, A, B, TW, TH, true>(p, lds, ox0, oy0);
    else
        group_body<CH, A, B, TW, TH, false>(p, lds, ox0, oy0);
}

// Groups without a window stage: one pass over the pixels.  Point stages need
// no coordinates, so a frame is a flat array of W*H pixels; each thread takes
// 4 consecutive pixels with vector loads and stores when the frame size is a
// multiple of 4 and the buffers are 16-byte aligned (every plane then starts
// 16-byte aligned for floats and 4-byte aligned for bytes), else one pixel.
template <int CH, int A, int B, int V>
__device__ __forceinline__ void stream_px(const SegParams& p, size_t plane, int t, size_t i)
{
    constexpr OpInfo oa = op_info(chain_op(CH, A));
    constexpr OpInfo ob = op_info(chain_op(CH, B));
    constexpr bool TEMPORAL = chain_op(CH, B) == FZ_OP_FRAMEDIFF;
    constexpr int E = pw_end(CH, A, B);
    const size_t vol = plane * p.T;
    float v[V][3];
    auto load = [&](int tt, float (&dst)[V][3]) {
        const size_t off = (size_t)tt * plane + i;
        if constexpr (oa.op == FZ_OP_RGB2GRAY) {
            const uint8_t* s = (const uint8_t*)p.in + 3 * off;
            if constexpr (V == 4) {
                const uint3 w = *(const uint3*)s;
                const uint32_t b[3] = {w.x, w.y, w.z};
#pragma unroll
                for (int k = 0; k < 12; ++k) dst[k / 3][k % 3] = (float)((b[k / 4] >> (8 * (k % 4))) & 255u);
            } else {
                for (int c = 0; c < 3; ++c) dst[0][c] = (float)s[c];
            }
        } else if constexpr (oa.in_dt == FZ_U8) {
            const uint8_t* s = (const uint8_t*)p.in + off;
            if constexpr (V == 4) {
                const uint32_t w = *(const uint32_t*)s;
#pragma unroll
                for (int k = 0; k < 4; ++k) dst[k][0] = (float)((w >> (8 * k)) & 255u);
            } else {
                dst[0][0] = (float)s[0];
            }
        } else {
#pragma unroll
            for (int c = 0; c < oa.in_ch; ++c) {
                const float* s = (const float*)p.in + c * vol + off;
                if constexpr (V == 4) {
                    const float4 w = *(const float4*)s;
                    dst[0][c] = w.x;
                    dst[1][c] = w.y;
                    dst[2][c] = w.z;
                    dst[3][c] = w.w;
                } else {
                    dst[0][c] = s[0];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) point_run<CH, A, E>(dst[k], p);
    };
    load(t, v);
    if constexpr (TEMPORAL) {
        float u[V][3];
        load(t > 0 ? t - 1 : 0, u);
#pragma unroll
        for (int k = 0; k < V; ++k) v[k][0] = (float)framediff((uint32_t)v[k][0], (uint32_t)u[k][0]);
    }
    const size_t off = (size_t)t * plane + i;
    if constexpr (ob.out_dt == FZ_U8) {
        uint8_t* d = (uint8_t*)p.out + off;
        if constexpr (V == 4) {
            uint32_t w = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) w |= ((uint32_t)v[k][0] & 255u) << (8 * k);
            *(uint32_t*)d = w;
        } else {
            d[0] = (uint8_t)(uint32_t)v[0][0];
        }
    } else {
#pragma unroll
        for (int c = 0; c < ob.out_ch; ++c) {
            float* d = (float*)p.out + c * vol + off;
            if constexpr (V == 4)
                *(float4*)d = make_float4(v[0][c], v[1][c], v[2][c], v[3][c]);
            else
                d[0] = v[0][c];
        }
    }
}

template <int CH, int A, int B>
__global__ __launch_bounds__(BLOCK_THREADS) void k_stream(SegParams p)
{
    const size_t plane = (size_t)p.W * p.H;
    const int t = blockIdx.y;
    const size_t stride = (size_t)gridDim.x * BLOCK_THREADS;
    const bool aligned = (((uintptr_t)p.in | (uintptr_t)p.out) & 15u) == 0;
    if (plane % 4 == 0 && aligned) {
        const size_t n4 = plane / 4;
        for (size_t q = (size_t)blockIdx.x * BLOCK_THREADS + threadIdx.x; q < n4; q += stride)
            stream_px<CH, A, B, 4>(p, plane, t, 4 * q);
    } else {
        for (size_t i = (size_t)blockIdx.x * BLOCK_THREADS + threadIdx.x; i < plane; i += stride)
            stream_px<CH, A, B, 1>(p, plane, t, i);
    }
}

// Launch group A..B of chain CH with tile index `tile`.
template <int CH, int A, int B>
hipError_t launch_group(const SegParams& p, int tile, hipStream_t s)
{
    if constexpr (A > B || B >= chain_len(CH) || A < 0) {
        return hipErrorInvalidValue;
    } else if constexpr (!group_has_window(CH, A, B)) {
        const int n = p.W * p.H;
        const int per = n % 4 == 0 ? n / 4 : n;
        int bx = (per + BLOCK_THREADS - 1) / BLOCK_THREADS;
        if (bx > 65535) bx = 65535;
        hipLaunchKernelGGL((k_stream<CH, A, B>), dim3(bx, p.T), dim3(BLOCK_THREADS), 0, s, p);
        return hipGetLastError();
    } else {
        auto go = [&](auto kern, int tw, int th) {
            dim3 grid((p.W + tw - 1) / tw, (p.H + th - 1) / th, (p.T + p.tpb - 1) / p.tpb);
            hipLaunchKernelGGL(kern, grid, dim3(BLOCK_THREADS), 0, s, p);
            return hipGetLastError();
        };
        switch (tile) {
        case 0: return go(k_group<CH, A, B, tile_w(0), tile_h(0)>, tile_w(0), tile_h(0));
        case 1: return go(k_group<CH, A, B, tile_w(1), tile_h(1)>, tile_w(1), tile_h(1));
        case 2: return go(k_group<CH, A, B, tile_w(2), tile_h(2)>, tile_w(2), tile_h(2));
        default: return hipErrorInvalidValue;
        }
    }
}

using LaunchFn = hipError_t (*)(const SegParams&, int, hipStream_t);

}  // namespace fz
