// Per-pixel arithmetic of every stage, in one fixed operation order.
//
// Every kernel variant (one kernel per stage, any fused group, the batched
// launch) calls these functions and the library is built with
// -ffp-contract=off, so a pixel's FP32 result does not depend on the
// partition: fusion changes where intermediates live, not what is computed
// (Sec. V-B: the fused kernel executes the same instructions, Algorithm 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fz {

// Point op: integer BT.601 luma, round half up.  (299R + 587G + 114B + 500)
// is at most 255500, and the division by the constant 1000 is exact integer
// division.
__device__ __forceinline__ uint32_t rgb2gray(uint32_t r, uint32_t g, uint32_t b)
{
    // x = 299R + 587G + 114B + 500 <= 255500 < 2^24, so 24-bit multiplies are
    // exact (full rate, where 32-bit multiplies issue at a quarter of it).
    const uint32_t x = __umul24(299u, r) + __umul24(587u, g) + __umul24(114u, b) + 500u;
    // floor(x / 1000) is the high word of x * ceil(2^32 / 1000) = x * 0x418938
    // for every x <= 255500 (checked exhaustively); both factors are below
    // 2^24, so the 24-bit multiply-high gives it in one instruction.
    uint32_t q;
    asm("v_mul_hi_u32_u24 %0, 0x418938, %1" : "=v"(q) : "v"(x));
    return q;
}

// Symmetric 5-tap weighted sum: w2*(x-2 + x+2) + w1*(x-1 + x+1) + w0*x0.
struct Gauss5W {
    float w0, w1, w2;
};
__device__ __forceinline__ float gauss5_taps(const Gauss5W& w, float m2, float m1, float c, float p1, float p2)
{
    float acc = w.w2 * (m2 + p2);
    acc = __builtin_fmaf(w.w1, m1 + p1, acc);
    return __builtin_fmaf(w.w0, c, acc);
}

// Unnormalised Sobel, evaluated column first.  Per column x:
//   sv(x) = 2 G(y,x) + (G(y-1,x) + G(y+1,x))      (vertical 1-2-1 smoothing)
//   e(x)  = G(y+1,x) - G(y-1,x)                    (vertical difference)
// then Ix = sv(x+1) - sv(x-1) and Iy = 2 e(x) + (e(x-1) + e(x+1)).
__device__ __forceinline__ float sobel_sv(float gm, float g0, float gp) { return __builtin_fmaf(2.0f, g0, gm + gp); }
__device__ __forceinline__ float sobel_e(float gm, float gp) { return gp - gm; }
__device__ __forceinline__ float sobel_ix(float sv_left, float sv_right) { return sv_right - sv_left; }
__device__ __forceinline__ float sobel_iy(float e_left, float e0, float e_right)
{
    return __builtin_fmaf(2.0f, e0, e_left + e_right);
}
// The same from a 3x3 window g[row][col] (rows y-1..y+1, columns x-1..x+1).
__device__ __forceinline__ void sobel3(const float g[3][3], float& ix, float& iy)
{
    ix = sobel_ix(sobel_sv(g[0][0], g[1][0], g[2][0]), sobel_sv(g[0][2], g[1][2], g[2][2]));
    iy = sobel_iy(sobel_e(g[0][0], g[2][0]), sobel_e(g[0][1], g[2][1]), sobel_e(g[0][2], g[2][2]));
}

__device__ __forceinline__ float gradmag(float ix, float iy)
{
    return __builtin_sqrtf(__builtin_fmaf(ix, ix, iy * iy));
}

__device__ __forceinline__ void products(float ix, float iy, float& pxx, float& pxy, float& pyy)
{
    pxx = ix * ix;
    pxy = ix * iy;
    pyy = iy * iy;
}

// Five-term sum: the two leading pairs, then the fifth term.  Neighbouring
// windows of a row then share their pair sums (the row kernel adds each pair
// of adjacent columns once).
__device__ __forceinline__ float sum5(float a, float b, float c, float d, float e)
{
    return ((a + b) + (c + d)) + e;
}

__device__ __forceinline__ float harris(float sxx, float sxy, float syy, float k)
{
    float det = __builtin_fmaf(sxx, syy, -(sxy * sxy));
    float tr = sxx + syy;
    return __builtin_fmaf(-k, tr * tr, det);
}

__device__ __forceinline__ float threshold(float v, float thr) { return v >= thr ? v : 0.0f; }

__device__ __forceinline__ float max3(float a, float b, float c) { return __builtin_fmaxf(__builtin_fmaxf(a, b), c); }

// 3x3 suppression decision given the centre and the window maximum.
__device__ __forceinline__ uint32_t nms_keep(float c, float wmax) { return (c > 0.0f && c >= wmax) ? 255u : 0u; }

__device__ __forceinline__ uint32_t framediff(uint32_t cur, uint32_t prev) { return cur > prev ? cur - prev : prev - cur; }

}  // namespace fz
