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
template <bool STENCIL, int RX, int RY>
__device__ __forceinline__ void windowq(const float* src, int RW, int base, const float* w, float (&acc)[GQ])
{
#pragma unroll
    for (int k = 0; k < GQ; ++k) acc[k] = 0.0f;
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
    case 0: windowq<STENCIL, RX, 0>(src, RW, base, w, acc); break;
    case 1: windowq<STENCIL, RX, 1>(src, RW, base, w, acc); break;
    case 2: windowq<STENCIL, RX, 2>(src, RW, base, w, acc); break;
    default: windowq<STENCIL, RX, 3>(src, RW, base, w, acc); break;
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

template <int TW, int TH>
static hipError_t launch_tile(const GParams& gp, int lds, hipStream_t s)
{
    if (lds > 65536) {  // allow the dynamic LDS beyond 64 KB (the CU has 160 KB)
        hipError_t e = hipFuncSetAttribute((const void*)k_gtile<TW, TH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           163840);
        if (e != hipSuccess) return e;
    }
    const long long blocks = (long long)gp.tiles_x * gp.tiles_y * gp.T;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    k_gtile<TW, TH><<<dim3((unsigned)blocks), dim3(BLOCK_THREADS), lds, s>>>(gp);
    return hipGetLastError();
}

int launch_generic(const fz_plan& p, const Segment& g, const void* in, void* out, void* stream)
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
    int nw = 0;
    for (int j = g.first; j <= g.last; ++j) {
        const fz_stage& st = p.stages[j];
        GStage& d = gp.st[j - g.first];
        d.kind = st.op == FZ_OP_POINT ? G_POINT : (st.op == FZ_OP_STENCIL ? G_STENCIL : G_BOX);
        d.rx = st.rx;
        d.ry = st.ry;
        d.pk = (int)st.param[0];
        d.a = st.param[1];
        d.b = st.param[2];
        if (d.kind == G_STENCIL) {
            const int cnt = (2 * st.rx + 1) * (2 * st.ry + 1);
            d.woff = nw;
            std::copy(p.gweights.begin() + p.gwoff[j], p.gweights.begin() + p.gwoff[j] + cnt, gp.w + nw);
            nw += cnt;
        }
    }
    if (g.engine == FZ_ENGINE_STREAM) {
        const size_t n = (size_t)p.W * p.H * p.T;
        const size_t want = (n + BLOCK_THREADS - 1) / BLOCK_THREADS;
        const unsigned blocks = (unsigned)std::min<size_t>(want, 256 * 32);
        k_gstream<<<dim3(blocks), dim3(BLOCK_THREADS), 0, s>>>(gp);
        return hipGetLastError();
    }
    gp.tiles_x = (p.W + g.tile_w - 1) / g.tile_w;
    gp.tiles_y = (p.H + g.tile_h - 1) / g.tile_h;
    switch (g.tile) {
    case 0: return launch_tile<tile_w(0), tile_h(0)>(gp, g.lds_bytes, s);
    case 1: return launch_tile<tile_w(1), tile_h(1)>(gp, g.lds_bytes, s);
    case 2: return launch_tile<tile_w(2), tile_h(2)>(gp, g.lds_bytes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fz
