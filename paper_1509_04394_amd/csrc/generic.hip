// Generic single-channel chains on the device.
//
// A group with a window stage runs as one LDS tile kernel (Algorithm 1): a
// workgroup loads the input box of its output tile, grown by the group's halo
// (the sums of the window radii, per axis), into LDS once, then runs the
// window stages one after another between two LDS buffers, each over the box
// that the later stages still need, and writes the last stage's tile to global
// memory.  Point stages never get a pass of their own: the ones before the
// first window stage run on the loaded values, the ones after a window stage
// on that stage's results before they are stored.  A group of point stages
// only is one streaming pass.
//
// The stage list and the stencil weights are kernel arguments (GParams); the
// loops over taps are uniform across the workgroup, so the weights are read
// with scalar loads.  Every window read clamps to the frame (replicate
// borders per stage).  The arithmetic order is fixed (stencil: row by row,
// each row left to right, fused multiply-adds from 0; window sum: each row
// left to right, rows top to bottom), so every tile shape and every partition
// gives the same bits.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "fz_internal.h"
#include "generic.h"

namespace fz {

__device__ __forceinline__ float gpoint(const GStage& s, float v)
{
    switch (s.pk) {
    case FZ_POINT_AFFINE: return fmaf(s.a, v, s.b);
    case FZ_POINT_ABS: return fabsf(v);
    case FZ_POINT_SQUARE: return v * v;
    case FZ_POINT_SQRTABS: return sqrtf(fabsf(v));
    default: return fminf(fmaxf(v, s.a), s.b);
    }
}

// Blocks are dealt to the 8 XCDs round-robin (block b on XCD b % 8).  Renumber
// them so that each XCD gets a contiguous run of tiles: neighbouring tiles,
// whose input boxes overlap by the halo, then share that XCD's L2.  A
// bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_contiguous(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, xcd = b & 7, slot = b >> 3;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + slot;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Quotient and remainder of e by a wavefront-uniform divisor d > 0 without an
// integer divide (which the hardware lacks): a single-precision estimate,
// then one correction step.  Exact for 0 <= e < 2^20 (a box has at most
// 40960 cells), where the estimate is off by at most one.
struct UDiv {
    int d;
    float inv;
    __device__ __forceinline__ explicit UDiv(int dd) : d(dd), inv(1.0f / (float)dd) {}
    __device__ __forceinline__ int quot(int e, int& rem) const
    {
        int q = (int)((float)e * inv);
        int r = e - q * d;
        if (r < 0) {
            --q;
            r += d;
        } else if (r >= d) {
            ++q;
            r -= d;
        }
        rem = r;
        return q;
    }
};

// GQ neighbouring cells of one row of a window stage whose whole input box
// lies inside the frame (no clamping): each input row is read once into
// registers, GQ + 2RX values, and every cell sums in the same order as the
// general path (rows top to bottom, each row left to right), so the bits are
// the same.  `base` is the box index of the first cell.  GQ is odd: the
// groups' first cells then lie GQ words apart from lane to lane, a stride
// coprime with the LDS bank count, so the lanes of a read or write fall on
// distinct banks (with four cells per thread, four lanes share each bank).
constexpr int GQ = 5;
// The window of GQ cells is added into acc, which the caller zeroes first (a
// stencil that looks back over several frames adds one frame after another).
template <bool STENCIL, int RX, int RY>
__device__ __forceinline__ void windowq_add(const float* src, int RW, int base, const float* w, float (&acc)[GQ])
{
#pragma unroll
    for (int v = -RY; v <= RY; ++v) {
        float x[GQ + 2 * RX];
        const int r0 = base + v * RW - RX;
#pragma unroll
        for (int q = 0; q < GQ + 2 * RX; ++q) x[q] = src[r0 + q];
        if constexpr (STENCIL) {
#pragma unroll
            for (int u = -RX; u <= RX; ++u) {
                const float wv = w[(v + RY) * (2 * RX + 1) + (u + RX)];
#pragma unroll
                for (int k = 0; k < GQ; ++k) acc[k] = fmaf(wv, x[k + u + RX], acc[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < GQ; ++k) {
                float h = 0.0f;
#pragma unroll
                for (int u = -RX; u <= RX; ++u) h = h + x[k + u + RX];
                acc[k] = acc[k] + h;
            }
        }
    }
}
template <bool STENCIL, int RX>
__device__ __forceinline__ void windowq_ry(int ry, const float* src, int RW, int base, const float* w,
                                           float (&acc)[GQ])
{
    switch (ry) {
    case 0: windowq_add<STENCIL, RX, 0>(src, RW, base, w, acc); break;
    case 1: windowq_add<STENCIL, RX, 1>(src, RW, base, w, acc); break;
    case 2: windowq_add<STENCIL, RX, 2>(src, RW, base, w, acc); break;
    default: windowq_add<STENCIL, RX, 3>(src, RW, base, w, acc); break;
    }
}
template <bool STENCIL>
__device__ __forceinline__ void windowq_r(int rx, int ry, const float* src, int RW, int base, const float* w,
                                          float (&acc)[GQ])
{
    switch (rx) {
    case 0: windowq_ry<STENCIL, 0>(ry, src, RW, base, w, acc); break;
    case 1: windowq_ry<STENCIL, 1>(ry, src, RW, base, w, acc); break;
    case 2: windowq_ry<STENCIL, 2>(ry, src, RW, base, w, acc); break;
    default: windowq_ry<STENCIL, 3>(ry, src, RW, base, w, acc); break;
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(BLOCK_THREADS) void k_gtile(const GParams p)
{
    extern __shared__ float glds[];
    const int RW = TW + 2 * p.hx, RH = TH + 2 * p.hy;
    float* src = glds;
    float* dst = glds + RW * RH;

    int b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int tx = b % p.tiles_x;
    b /= p.tiles_x;
    const int ty = b % p.tiles_y;
    const int t = b / p.tiles_y;
    const int ox = tx * TW - p.hx, oy = ty * TH - p.hy;  // frame position of the box's first cell
    const size_t fbase = (size_t)t * p.W * p.H;
    // the whole input box inside the frame: no read needs clamping
    const bool interior = ox >= 0 && oy >= 0 && ox + RW <= p.W && oy + RH <= p.H;

    int lead = 0;
    while (lead < p.n && p.st[lead].kind == G_POINT) ++lead;

    // the input box; cells outside the frame are never read (reads clamp)
    const UDiv by_rw(RW);
    for (int e = threadIdx.x; e < RW * RH; e += BLOCK_THREADS) {
        int lx;
        const int ly = by_rw.quot(e, lx);
        const int gx = ox + lx, gy = oy + ly;
        if (gx < 0 || gx >= p.W || gy < 0 || gy >= p.H) continue;
        const size_t gi = fbase + (size_t)gy * p.W + gx;
        float v = p.in_u8 ? (float)((const uint8_t*)p.in)[gi] : ((const float*)p.in)[gi];
        for (int j = 0; j < lead; ++j) v = gpoint(p.st[j], v);
        src[e] = v;
    }
    __syncthreads();

    int i = lead, hx = p.hx, hy = p.hy;
    while (i < p.n) {
        const GStage s = p.st[i];
        int j = i + 1;
        while (j < p.n && p.st[j].kind == G_POINT) ++j;
        const bool last = j == p.n;
        const int ohx = hx - s.rx, ohy = hy - s.ry;        // halo still needed after this stage
        const int OW = TW + 2 * ohx, OH = TH + 2 * ohy;   // cells this stage computes
        const int bx = p.hx - ohx, by = p.hy - ohy;       // their first cell in box coordinates
        const int kw = 2 * s.rx + 1;
        if (interior) {
            // GQ neighbouring cells per thread; the last group of a row may
            // read up to GQ - 1 cells past it (into the next row or the padding)
            const int NQ = (OW + GQ - 1) / GQ;
            const float* w = p.w + s.woff;
            const UDiv by_nq(NQ);
            for (int e = threadIdx.x; e < NQ * OH; e += BLOCK_THREADS) {
                int qx;
                const int cy = by_nq.quot(e, qx), cx = qx * GQ;
                const int lx = bx + cx, ly = by + cy;
                float acc[GQ];
#pragma unroll
                for (int k = 0; k < GQ; ++k) acc[k] = 0.0f;
                if (s.kind == G_STENCIL)
                    windowq_r<true>(s.rx, s.ry, src, RW, ly * RW + lx, w, acc);
                else
                    windowq_r<false>(s.rx, s.ry, src, RW, ly * RW + lx, w, acc);
                const int nk = min(GQ, OW - cx);
#pragma unroll
                for (int k = 0; k < GQ; ++k) {
                    if (k >= nk) break;
                    float v = acc[k];
                    for (int q = i + 1; q < j; ++q) v = gpoint(p.st[q], v);
                    if (last)
                        p.out[fbase + (size_t)(oy + ly) * p.W + (ox + lx + k)] = v;
                    else
                        dst[ly * RW + lx + k] = v;
                }
            }
        } else {
            const UDiv by_ow(OW);
            for (int e = threadIdx.x; e < OW * OH; e += BLOCK_THREADS) {
                int cx;
                const int cy = by_ow.quot(e, cx);
                const int lx = bx + cx, ly = by + cy;
                const int gx = ox + lx, gy = oy + ly;
                if (gx < 0 || gx >= p.W || gy < 0 || gy >= p.H) continue;
                float acc = 0.0f;
                for (int v = -s.ry; v <= s.ry; ++v) {
                    // box index of the clamped cell (x, y) = (y - oy) * RW + (x - ox)
                    const int row = (clampi(gy + v, 0, p.H - 1) - oy) * RW - ox;
                    if (s.kind == G_STENCIL) {
                        const int w0 = s.woff + (v + s.ry) * kw + s.rx;
                        for (int u = -s.rx; u <= s.rx; ++u)
                            acc = fmaf(p.w[w0 + u], src[row + clampi(gx + u, 0, p.W - 1)], acc);
                    } else {
                        float h = 0.0f;
                        for (int u = -s.rx; u <= s.rx; ++u) h = h + src[row + clampi(gx + u, 0, p.W - 1)];
                        acc = acc + h;
                    }
                }
                for (int q = i + 1; q < j; ++q) acc = gpoint(p.st[q], acc);
                if (last)
                    p.out[fbase + (size_t)gy * p.W + gx] = acc;
                else
                    dst[ly * RW + lx] = acc;
            }
        }
        if (last) break;
        __syncthreads();
        float* tmp = src;
        src = dst;
        dst = tmp;
        hx = ohx;
        hy = ohy;
        i = j;
    }
}

// A group of point stages: one pass, each thread a run of pixels strided by
// the grid.
__global__ __launch_bounds__(BLOCK_THREADS) void k_gstream(const GParams p)
{
    const size_t n = (size_t)p.W * p.H * p.T;
    const size_t stride = (size_t)gridDim.x * BLOCK_THREADS;
    for (size_t i = (size_t)blockIdx.x * BLOCK_THREADS + threadIdx.x; i < n; i += stride) {
        float v = p.in_u8 ? (float)((const uint8_t*)p.in)[i] : ((const float*)p.in)[i];
        for (int j = 0; j < p.n; ++j) v = gpoint(p.st[j], v);
        p.out[i] = v;
    }
}

// ------------------------------------------------------------ temporal stages
//
// Table II's IIR filter is a point operation over several frames: per pixel,
// y[t] = a x[t] + (1 - a) y[t-1] with y[-1] := x[0].  It runs in double
// precision -- the state and fma(a, x, (1 - a) y_prev), with 1 - a exact in
// double for an f32 a -- and each output is rounded once to f32: in f32 the
// recursion's rounding errors would pile up over about 1/a frames (a = 0.05
// gave 1.1e-4 on a 0-255 scale).  A stencil
// may also look rt frames back (Table I's spatio-temporal class):
// out(t) = sum over tau = 0..rt (this frame first) of the frame t - tau
// window, frames before the first replicating the first; each frame's window
// is summed as the spatial stencil sums it, continuing one fused multiply-add
// chain.  Groups with such stages march through frames in order.

// One IIR step of the cell whose running state is *state (first: frame 0).
__device__ __forceinline__ float giir(const GStage& s, float v, double* state, bool first)
{
    const double a = (double)s.a, x = (double)v;
    const double prev = first ? x : *state;
    const double y = fma(a, x, (1.0 - a) * prev);
    *state = y;
    return (float)y;
}

// Point and IIR stages q0..q1-1 on one value of box cell `cell`.  Each stage
// descriptor is copied out of the kernel arguments first: a reference into
// them next to the IIR's LDS store made the compiler copy the whole argument
// block into scratch memory.
__device__ __forceinline__ float gtrail(const GParams& p, float* lds, int q0, int q1, float v, int cell, bool first)
{
    for (int q = q0; q < q1; ++q) {
        const GStage s = p.st[q];
        v = s.kind == G_IIR ? giir(s, v, (double*)(lds + s.buf) + cell, first) : gpoint(s, v);
    }
    return v;
}

// A group with a window stage and a temporal stage (an IIR, or a stencil that
// looks back): one workgroup owns an output tile and a run of tt frames and
// marches through frames t0 - ht .. t0 + tt - 1 in order (from frame 0 when the
// run starts within ht frames of it, and always from frame 0 for an IIR, whose
// runs are the whole clip).  Per frame it loads the input box once and runs the
// stages as the tile kernel does; a stencil that looks back reads its earlier
// input frames from a ring in LDS, an IIR keeps its state per box cell in
// LDS (layout: march_layout).  The frames before t0 only fill the rings: a
// stage skips a frame whose ring is not yet full, and nothing is stored before
// t0.  Every stage evaluates exactly as in the tile kernel, so the bits do not
// depend on the partition, the tile or the frame run.
template <int TW, int TH>
__global__ __launch_bounds__(BLOCK_THREADS) void k_gmarch(const GParams p)
{
    extern __shared__ float glds[];
    const int RW = TW + 2 * p.hx, RH = TH + 2 * p.hy, CELLS = RW * RH;
    int b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int tx = b % p.tiles_x;
    b /= p.tiles_x;
    const int ty = b % p.tiles_y;
    const int t0 = (b / p.tiles_y) * p.tt;
    const int t1 = min(p.T, t0 + p.tt);
    const int fs = max(0, t0 - p.ht);  // first frame marched
    const int ox = tx * TW - p.hx, oy = ty * TH - p.hy;
    const size_t P = (size_t)p.W * p.H;
    const bool interior = ox >= 0 && oy >= 0 && ox + RW <= p.W && oy + RH <= p.H;

    int lead = 0;
    while (lead < p.n && !g_is_window(p.st[lead].kind)) ++lead;
    const UDiv by_rw(RW);

    if (p.ck_n > 0 && t0 > 0) {
        // the leading IIRs resume from the first pass's state after frame t0 - 1
        const double* ck = p.ckpt + (size_t)(t0 / p.tt - 1) * p.ck_n * P;
        for (int e = threadIdx.x; e < CELLS; e += BLOCK_THREADS) {
            int lx;
            const int ly = by_rw.quot(e, lx);
            const int gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gx >= p.W || gy < 0 || gy >= p.H) continue;
            int k = 0;
            for (int j = 0; j < lead; ++j) {
                const GStage sj = p.st[j];
                if (sj.kind != G_IIR) continue;
                ((double*)(glds + sj.buf))[e] = ck[(size_t)k * P + (size_t)gy * p.W + gx];
                ++k;
            }
        }
        __syncthreads();
    }

    for (int f = fs; f < t1; ++f) {
        const bool first = f == 0;
        const size_t fbase = (size_t)f * P;
        {
            const GStage& s0 = p.st[lead];
            float* dst = glds + s0.buf + (f % s0.slots) * CELLS;
            for (int e = threadIdx.x; e < CELLS; e += BLOCK_THREADS) {
                int lx;
                const int ly = by_rw.quot(e, lx);
                const int gx = ox + lx, gy = oy + ly;
                if (gx < 0 || gx >= p.W || gy < 0 || gy >= p.H) continue;
                const size_t gi = fbase + (size_t)gy * p.W + gx;
                const float v = p.in_u8 ? (float)((const uint8_t*)p.in)[gi] : ((const float*)p.in)[gi];
                dst[e] = gtrail(p, glds, 0, lead, v, e, first);
            }
        }
        __syncthreads();

        int i = lead, hx = p.hx, hy = p.hy, back = 0;
        while (true) {
            const GStage s = p.st[i];
            int j = i + 1;
            while (j < p.n && !g_is_window(p.st[j].kind)) ++j;
            const bool last = j == p.n;
            back += s.rt;
            const int ohx = hx - s.rx, ohy = hy - s.ry;
            const int OW = TW + 2 * ohx, OH = TH + 2 * ohy;
            const int bx = p.hx - ohx, by = p.hy - ohy;
            // this stage's input ring holds frames f - rt .. f (replicated before frame 0)
            const bool ready = fs == 0 || f >= fs + back;
            if (ready && (!last || f >= t0)) {
                float* dst = last ? nullptr : glds + p.st[j].buf + (f % p.st[j].slots) * CELLS;
                const int nw = (2 * s.rx + 1) * (2 * s.ry + 1);
                if (interior) {
                    const int NQ = (OW + GQ - 1) / GQ;
                    const UDiv by_nq(NQ);
                    for (int e = threadIdx.x; e < NQ * OH; e += BLOCK_THREADS) {
                        int qx;
                        const int cy = by_nq.quot(e, qx), cx = qx * GQ;
                        const int lx = bx + cx, ly = by + cy;
                        float acc[GQ];
#pragma unroll
                        for (int k = 0; k < GQ; ++k) acc[k] = 0.0f;
                        for (int tau = 0; tau <= s.rt; ++tau) {
                            const float* src = glds + s.buf + (max(f - tau, 0) % s.slots) * CELLS;
                            if (s.kind == G_STENCIL)
                                windowq_r<true>(s.rx, s.ry, src, RW, ly * RW + lx, p.w + s.woff + tau * nw, acc);
                            else
                                windowq_r<false>(s.rx, s.ry, src, RW, ly * RW + lx, nullptr, acc);
                        }
                        const int nk = min(GQ, OW - cx);
#pragma unroll
                        for (int k = 0; k < GQ; ++k) {
                            if (k >= nk) break;
                            const float v = gtrail(p, glds, i + 1, j, acc[k], ly * RW + lx + k, first);
                            if (last)
                                p.out[fbase + (size_t)(oy + ly) * p.W + (ox + lx + k)] = v;
                            else
                                dst[ly * RW + lx + k] = v;
                        }
                    }
                } else {
                    const int kw = 2 * s.rx + 1;
                    const UDiv by_ow(OW);
                    for (int e = threadIdx.x; e < OW * OH; e += BLOCK_THREADS) {
                        int cx;
                        const int cy = by_ow.quot(e, cx);
                        const int lx = bx + cx, ly = by + cy;
                        const int gx = ox + lx, gy = oy + ly;
                        if (gx < 0 || gx >= p.W || gy < 0 || gy >= p.H) continue;
                        float acc = 0.0f;
                        for (int tau = 0; tau <= s.rt; ++tau) {
                            const float* src = glds + s.buf + (max(f - tau, 0) % s.slots) * CELLS;
                            for (int v = -s.ry; v <= s.ry; ++v) {
                                const int row = (clampi(gy + v, 0, p.H - 1) - oy) * RW - ox;
                                if (s.kind == G_STENCIL) {
                                    const int w0 = s.woff + tau * nw + (v + s.ry) * kw + s.rx;
                                    for (int u = -s.rx; u <= s.rx; ++u)
                                        acc = fmaf(p.w[w0 + u], src[row + clampi(gx + u, 0, p.W - 1)], acc);
                                } else {
                                    float h = 0.0f;
                                    for (int u = -s.rx; u <= s.rx; ++u) h = h + src[row + clampi(gx + u, 0, p.W - 1)];
                                    acc = acc + h;
                                }
                            }
                        }
                        const float v = gtrail(p, glds, i + 1, j, acc, ly * RW + lx, first);
                        if (last)
                            p.out[fbase + (size_t)gy * p.W + gx] = v;
                        else
                            dst[ly * RW + lx] = v;
                    }
                }
            }
            if (last) break;
            __syncthreads();
            hx = ohx;
            hy = ohy;
            i = j;
        }
        __syncthreads();  // the next frame's load reuses the buffers
    }
}

// A group of point and IIR stages only: each thread owns PX neighbouring
// pixels and marches through every frame in order; D frames are loaded before
// any is processed, so D loads per thread are in flight at once.  With ONE
// (the group has a single IIR) its states are PX registers; otherwise the
// IIR states (doubles) live in LDS, PX per thread and IIR stage (GStage::buf
// is the stage's offset there, in doubles): registers indexed by a stage
// number only known at run time would have gone to scratch memory.
//
// With CKPT, the kernel is the first pass of a checkpointed group: it runs
// the group's leading point and IIR stages only (p.n of them), stores no
// output, and after the last frame of every frame run but the last writes
// each IIR's state to p.ckpt[run][IIR][pixel].
template <int PX, int D, bool CKPT, bool ONE, bool RAW = false>
__global__ __launch_bounds__(BLOCK_THREADS) void k_gstream_t(const GParams p)
{
    extern __shared__ double gstate[];
    double rstate[PX];  // ONE: the IIR's states
#pragma unroll
    for (int k = 0; k < PX; ++k) rstate[k] = 0.0;
    const size_t P = (size_t)p.W * p.H;
    const size_t i0 = ((size_t)blockIdx.x * BLOCK_THREADS + threadIdx.x) * PX;
    if (i0 >= P) return;  // no barrier below
    for (int t = 0; t < p.T; t += D) {
        // RAW (u8 input, four pixels): the D frames' bytes stay packed, one
        // register per frame, so many frames can be in flight
        float v[RAW ? 1 : D][PX];
        uint32_t raw[RAW ? D : 1];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (t + d >= p.T) break;
            const size_t gi = (size_t)(t + d) * P + i0;
            if constexpr (RAW) {
                raw[d] = *(const uint32_t*)((const uint8_t*)p.in + gi);
            } else if constexpr (PX == 4) {
                if (p.in_u8) {
                    const uchar4 q = *(const uchar4*)((const uint8_t*)p.in + gi);
                    v[d][0] = q.x;
                    v[d][1] = q.y;
                    v[d][2] = q.z;
                    v[d][3] = q.w;
                } else {
                    const float4 q = *(const float4*)((const float*)p.in + gi);
                    v[d][0] = q.x;
                    v[d][1] = q.y;
                    v[d][2] = q.z;
                    v[d][3] = q.w;
                }
            } else {
                v[d][0] = p.in_u8 ? (float)((const uint8_t*)p.in)[gi] : ((const float*)p.in)[gi];
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (t + d >= p.T) break;
            float w[PX];
#pragma unroll
            for (int k = 0; k < PX; ++k) w[k] = RAW ? (float)((raw[RAW ? d : 0] >> (8 * k)) & 255u) : v[RAW ? 0 : d][k];
            const bool first = t + d == 0;
            const bool save = CKPT && (t + d + 1) % p.tt == 0 && t + d + 1 < p.T;
            int n_iir = 0;
            for (int j = 0; j < p.n; ++j) {
                const GStage s = p.st[j];
                if (s.kind == G_IIR) {
                    double* sp = ONE ? rstate : gstate + s.buf + threadIdx.x * PX;
                    const double a = (double)s.a;
#pragma unroll
                    for (int k = 0; k < PX; ++k) {
                        const double x = (double)w[k];
                        const double prev = ONE ? rstate[k] : sp[k];
                        const double y = fma(a, x, (1.0 - a) * (first ? x : prev));
                        if (ONE)
                            rstate[k] = y;
                        else
                            sp[k] = y;
                        w[k] = (float)y;
                    }
                    if (save) {
                        double* ck = (double*)p.ckpt + ((size_t)((t + d + 1) / p.tt - 1) * p.ck_n + n_iir) * P + i0;
#pragma unroll
                        for (int k = 0; k < PX; ++k) ck[k] = ONE ? rstate[k] : sp[k];
                    }
                    ++n_iir;
                } else {
#pragma unroll
                    for (int k = 0; k < PX; ++k) w[k] = gpoint(s, w[k]);
                }
            }
            if constexpr (!CKPT) {
                const size_t gi = (size_t)(t + d) * P + i0;
                if constexpr (PX == 4)
                    *(float4*)(p.out + gi) = make_float4(w[0], w[1], w[2], w[3]);
                else
                    p.out[gi] = w[0];
            }
        }
    }
}

template <typename K>
static hipError_t allow_lds(K kernel, int lds)
{
    if (lds <= 65536) return hipSuccess;
    // dynamic LDS beyond 64 KB (the CU has 160 KB)
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
}

template <int TW, int TH>
static hipError_t launch_tile(const GParams& gp, int lds, bool march, int nchunks, hipStream_t s)
{
    const long long blocks = (long long)gp.tiles_x * gp.tiles_y * (march ? nchunks : gp.T);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipError_t e;
    if (march) {
        if ((e = allow_lds(k_gmarch<TW, TH>, lds)) != hipSuccess) return e;
        k_gmarch<TW, TH><<<dim3((unsigned)blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    } else {
        if ((e = allow_lds(k_gtile<TW, TH>, lds)) != hipSuccess) return e;
        k_gtile<TW, TH><<<dim3((unsigned)blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    }
    return hipGetLastError();
}

// Launch a group of point and IIR stages through k_gstream_t (the whole group,
// or with CKPT the first pass of a checkpointed group).
template <bool CKPT>
static hipError_t launch_stream_t(GParams gp, const void* in, size_t P, hipStream_t s)
{
    int n_iir = 0;
    for (int j = 0; j < gp.n; ++j) n_iir += gp.st[j].kind == G_IIR ? 1 : 0;
    const bool one = n_iir == 1;
    // four pixels per thread where aligned; with one IIR on u8 input (its
    // states in registers, the input bytes kept packed) 32 frames are loaded
    // ahead: every thread marches all frames in order, so the kernel lives on
    // the bytes in flight, and a pixel per thread (64-byte pieces of frames
    // far apart) read at a fraction of the bandwidth
    const bool vec = P % 4 == 0 && ((uintptr_t)in % (gp.in_u8 ? 4 : 16)) == 0 &&
                     (CKPT || ((uintptr_t)gp.out % 16) == 0);
    const int px = vec ? 4 : 1;
    n_iir = 0;
    for (int j = 0; j < gp.n; ++j)
        if (gp.st[j].kind == G_IIR) gp.st[j].buf = (n_iir++) * BLOCK_THREADS * px;
    const int lds = one ? 0 : n_iir * BLOCK_THREADS * px * 8;  // doubles; a 4-pixel run with 16 IIRs: 128 KB
    hipError_t e = hipSuccess;
    if (lds > 65536) e = vec ? allow_lds(k_gstream_t<4, 8, CKPT, false>, lds) : allow_lds(k_gstream_t<1, 8, CKPT, false>, lds);
    if (e != hipSuccess) return e;
    const size_t threads = P / px;
    const unsigned blocks = (unsigned)((threads + BLOCK_THREADS - 1) / BLOCK_THREADS);
    if (vec && one && gp.in_u8)
        k_gstream_t<4, 32, CKPT, true, true><<<dim3(blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    else if (vec && one)
        k_gstream_t<4, 8, CKPT, true><<<dim3(blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    else if (vec)
        k_gstream_t<4, 8, CKPT, false><<<dim3(blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    else if (one)
        k_gstream_t<1, 8, CKPT, true><<<dim3(blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    else
        k_gstream_t<1, 8, CKPT, false><<<dim3(blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    return hipGetLastError();
}

size_t ckpt_bytes(const fz_plan& p, const Segment& g)
{
    if (!p.generic || !g.ckpt || g.tpb <= 0) return 0;
    GStage st[G_MAX_STAGES];
    g_stage_list(p.stages.data(), g.first, g.last, st);
    const int n_iir = g_ckpt_iirs(st, g.last - g.first + 1);
    const size_t runs = (size_t)(p.T + g.tpb - 1) / g.tpb;
    return runs > 1 ? (runs - 1) * n_iir * (size_t)p.W * p.H * sizeof(double) : 0;
}

int launch_generic(const fz_plan& p, const Segment& g, const void* in, void* out, void* ckpt, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    GParams gp{};
    gp.in = in;
    gp.out = (float*)out;
    gp.W = p.W;
    gp.H = p.H;
    gp.T = p.T;
    gp.in_u8 = p.stages[g.first].in_dtype == FZ_U8;
    gp.n = g.last - g.first + 1;
    gp.hx = g.halo;
    gp.hy = g.halo_y;
    if (gp.n > G_MAX_STAGES) return hipErrorInvalidValue;
    const int need = g_stage_list(p.stages.data(), g.first, g.last, gp.st);
    if (need > G_MAX_WEIGHTS) return hipErrorInvalidValue;  // the planner never forms such a group
    int nw = 0;
    for (int j = g.first; j <= g.last; ++j) {
        GStage& d = gp.st[j - g.first];
        if (d.kind != G_STENCIL) continue;
        const int cnt = (2 * d.rx + 1) * (2 * d.ry + 1) * (d.rt + 1);
        d.woff = nw;
        std::copy(p.gweights.begin() + p.gwoff[j], p.gweights.begin() + p.gwoff[j] + cnt, gp.w + nw);
        nw += cnt;
    }
    bool has_iir = false;
    const bool temporal = g_temporal(gp.st, gp.n, &has_iir, &gp.ht);
    const size_t P = (size_t)p.W * p.H;
    if (g.engine == FZ_ENGINE_STREAM) {
        if (temporal) return launch_stream_t<false>(gp, in, P, s);  // point and IIR stages, all frames
        const size_t n = P * p.T;
        const size_t want = (n + BLOCK_THREADS - 1) / BLOCK_THREADS;
        const unsigned blocks = (unsigned)std::min<size_t>(want, 256 * 32);
        k_gstream<<<dim3(blocks), dim3(BLOCK_THREADS), 0, s>>>(gp);
        return hipGetLastError();
    }
    if (g.engine == FZ_ENGINE_JIT && !temporal) return launch_jit(p, g, in, out, nullptr, stream);
    gp.tiles_x = (p.W + g.tile_w - 1) / g.tile_w;
    gp.tiles_y = (p.H + g.tile_h - 1) / g.tile_h;
    int nchunks = 1;
    if (temporal) {
        gp.tt = g.tpb;
        if (gp.tt < 1 || (has_iir && !g.ckpt && gp.tt < p.T)) return hipErrorInvalidValue;
        nchunks = (p.T + gp.tt - 1) / gp.tt;
        if (g.ckpt && nchunks > 1) {
            // first pass: the leading point and IIR stages over every pixel, checkpoints only
            if (!ckpt) return hipErrorInvalidValue;
            gp.ck_n = g_ckpt_iirs(gp.st, gp.n);
            gp.ckpt = (const double*)ckpt;
            GParams g1 = gp;
            int lead = 0;
            while (lead < gp.n && !g_is_window(gp.st[lead].kind)) ++lead;
            g1.n = lead;
            g1.out = nullptr;
            const hipError_t e = launch_stream_t<true>(g1, in, P, s);
            if (e != hipSuccess) return e;
        }
        if (g.engine == FZ_ENGINE_JIT) return launch_jit(p, g, in, out, ckpt, stream);
        const int floats = march_layout(gp.st, gp.n, (g.tile_w + 2 * gp.hx) * (g.tile_h + 2 * gp.hy));
        if ((floats + GEN_PAD) * 4 != g.lds_bytes) return hipErrorInvalidValue;
    }
    switch (g.tile) {
    case 0: return launch_tile<tile_w(0), tile_h(0)>(gp, g.lds_bytes, temporal, nchunks, s);
    case 1: return launch_tile<tile_w(1), tile_h(1)>(gp, g.lds_bytes, temporal, nchunks, s);
    case 2: return launch_tile<tile_w(2), tile_h(2)>(gp, g.lds_bytes, temporal, nchunks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fz
