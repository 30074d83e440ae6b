// Row-marching fused kernel for the Harris chain (gray or RGB input,
// Gaussian 5x5 -> Sobel -> products -> 5x5 sums -> Harris -> threshold ->
// 3x3 suppression [-> frame difference]).
//
// Same computation as the LDS tile engine (same per-pixel expressions, so the
// outputs are identical bit for bit), organised for gfx950 wavefronts:
//   * a wavefront owns a strip of 64*K columns (K adjacent columns per lane)
//     of a band of rows of one frame and marches down the rows; every window
//     stage keeps the few rows it still needs in registers (rings of 2r+1
//     rows; the 5x5 window sums keep sums of row pairs instead, and share
//     the pair sums of neighbouring columns across lanes), so nothing is
//     staged in LDS and no barrier is needed;
//   * horizontal neighbours come from the adjacent lanes through DPP wave
//     shifts; a lane at the strip's edge receives its own edge value, which is
//     exactly the replicate border when the strip touches the frame edge (and a
//     don't-care halo value inside the frame, where the strips overlap by the
//     chain's horizontal halo);
//   * the row loop is unrolled by 15 (the least common multiple of the ring
//     sizes 3 and 5) so every ring slot is a fixed register;
//   * vertical replicate borders: when a stage produces the first row of the
//     frame it also writes it into the ring slots of the rows above, and after
//     the last row it copies it into the slots of the rows below, one slot per
//     iteration, once the consumer no longer needs the slot's old row;
//   * the suppression mask feeds the frame difference through a per-wavefront
//     LDS row of previous-frame mask bits; a work item covers a run of frames.
//     The difference at the first frame of a run needs the mask of the frame
//     before it, which the item of the previous run computes anyway: the two
//     items meet at their shared frame boundary (see row_exchange) instead of
//     the later one computing that frame again.  Without the exchange buffers
//     an item first recomputes the frame before its run (one frame of
//     temporal halo).
// The input rows are prefetched two iterations ahead.
#pragma once

#include "engine.h"
#include "rowgeom.h"

namespace fz {

constexpr int ROW_UNROLL = 15;  // lcm of the ring sizes

struct RowParams {
    SegParams sp;
    int nstrips, nbands, nchunks, total;
    int strip_step;  // 64K - 2*ROW_HX
    int band_h;
    int tt;          // frames per work item
    // frame-boundary exchange (frame difference; null: recompute the frame
    // before each run instead): per boundary between runs c-1 and c of one
    // strip and band, two mask areas of band_h * K words (the earlier run's
    // last frame, the later run's first frame) and one arrival counter,
    // zeroed before the launch
    uint64_t* xmask;
    uint32_t* xcount;
};

// Value of the lane to the left (wave_shr:1) / right (wave_shl:1).  At a
// frame edge (EDGE) the edge lane keeps `edge`, its own edge column: the
// replicate border.  Inside the frame the edge lane is a halo lane whose value
// is never used, so it may read zero, which lets the compiler fold the shift
// into the instruction that consumes it.
template <bool EDGE>
__device__ __forceinline__ float dpp_from_left(float v, float edge)
{
    if constexpr (EDGE)
        return __int_as_float(
            __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xf, 0xf, false));
    else
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
template <bool EDGE>
__device__ __forceinline__ float dpp_from_right(float v, float edge)
{
    if constexpr (EDGE)
        return __int_as_float(
            __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xf, 0xf, false));
    else
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// e[0 .. K+2R) = this lane's columns x-R .. x+K-1+R of a row held K per lane.
// EL / ER: the strip's first / last column is the frame's.
template <int K, int R, bool EL, bool ER>
__device__ __forceinline__ void extend_row(const float (&v)[K], float (&e)[K + 2 * R])
{
    static_assert(R <= K, "neighbour lanes must hold the halo");
#pragma unroll
    for (int k = 0; k < K; ++k) e[R + k] = v[k];
#pragma unroll
    for (int i = 1; i <= R; ++i) {
        e[R - i] = dpp_from_left<EL>(v[K - i], v[0]);
        e[R + K - 1 + i] = dpp_from_right<ER>(v[i - 1], v[K - 1]);
    }
}

// Horizontal pass of the 5-wide window sum of a row held K per lane:
// s[k] = sum5(e[k], ..., e[k+4]) over the extended row e = extend_row<K, 2>(v),
// computed from pair sums p[j] = e[j] + e[j+1].  Window k needs p[k], p[k+2]
// and e[k+4]; each pair of adjacent columns is added once, by the lane that
// holds its right column, and a lane reads its neighbours' pairs through DPP
// shifts: p[0] is the left lane's p[K] and p[K+1] the right lane's p[1].  At
// a frame edge the shifted pair of the edge lane is the sum of its own edge
// column with itself, which is what the replicate border gives.  Same bits as
// sum5 on extend_row's output.
template <int K, bool EL, bool ER>
__device__ __forceinline__ void box5_row(const float (&v)[K], float (&s)[K])
{
    static_assert(K >= 2, "two or more columns per lane");
    float p[K + 2];
    p[1] = dpp_from_left<EL>(v[K - 1], v[0]) + v[0];  // straddles the left lane boundary
#pragma unroll
    for (int j = 2; j <= K; ++j) p[j] = v[j - 2] + v[j - 1];
    p[0] = dpp_from_left<EL>(p[K], p[1]);  // at the left frame edge p[1] = v[0] + v[0]
    p[K + 1] = dpp_from_right<ER>(p[1], ER ? v[K - 1] + v[K - 1] : 0.0f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float e4 = k + 2 < K ? v[k + 2] : dpp_from_right<ER>(v[k + 2 - K], v[K - 1]);
        s[k] = (p[k] + p[k + 2]) + e4;
    }
}

// Raw buffer over `bytes` bytes at `base`: a store whose offset is at or past
// `bytes` is dropped by the hardware, which lets every lane issue its store
// with no divergent branch (columns outside the strip's output range get an
// out-of-range offset).  Word 3 selects 32-bit raw access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}
constexpr int DROP = 0x7fffffff;  // an offset past any frame

template <int K>
__device__ __forceinline__ void copy_row(float (&d)[K], const float (&s)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = s[k];
}

// NB consecutive input bytes kept as loaded: whole dwords, then a short,
// then a byte.  The short and the byte keep their 16- and 8-bit types so that
// their zero extension happens where they are used, not right after the
// load (an operation on a loaded register makes the wavefront wait for the
// load).
template <int NB>
struct RawRow {
    static constexpr int ND = NB / 4;
    uint32_t d[ND > 0 ? ND : 1];
    uint16_t h;  // bytes 4*ND, 4*ND+1 when NB % 4 >= 2
    uint8_t y;   // the last byte when NB is odd
};

template <int K, bool RGB>
struct RowState {
    static constexpr int NB = RGB ? 3 * K : K;  // input bytes per lane and row
    float h[5][K];     // Gaussian horizontal pass
    float g[3][K];     // Gaussian output
    float bp[3][K];    // window-sum horizontal pass of the previous row, 3 channels
    float q[3][3][K];  // pairs of consecutive horizontal-pass rows, q_r = b_r + b_(r+1)
    float rt[3][K];    // thresholded response
    float m[3][K];     // 3-wide horizontal maximum of rt
    RawRow<NB> raw[3];  // input rows, two loaded ahead
};

struct RowCtx {
    const uint8_t* in_frame;  // frame t of the input
    uint8_t* out_frame;       // frame t of the output
    int W, Hf, x0, lane, y0, y1, t;
    int row_bytes;            // bytes per input row
    int lane_in, lane_out;    // byte offset of this lane's first column in an input / output row
    bool real;                // frame t is one of the item's own frames (feature points)
    bool store;               // its output is written now (not at a frame boundary exchange)
    uint32_t valid;           // bit k: column k of this lane is an output column of the strip
    int lo_in, hi_in, lo_g, hi_g, lo_s, hi_s, lo_b, hi_b;
    // iteration j computes a stage's row iff (unsigned)(j - j*) < n*: the rows
    // [lo, hi) of each stage mapped to iterations (row = y0 - 6 + j - lag)
    int jp, np_, ji, ni, jg, ng, js, ns, jq, nq, jb, nb, jn, nn;
    uint8_t* prev;            // LDS previous-frame mask bits of this wavefront (DIFF)
};

// NB consecutive bytes at byte offset voff + soff of buffer r into a RawRow:
// the fewest dword / short / byte loads; the bytes need not be aligned.  soff
// is wavefront-uniform (a scalar register), voff the lane's own offset, so
// the address needs no per-lane arithmetic.  byte_of<NB, I>(w) extracts byte
// I; keeping the bytes packed holds a row of 6 RGB bytes in 2 registers
// instead of 6.
template <int NB>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t r, int voff, int soff, RawRow<NB>& w)
{
    constexpr int D = NB / 4;
#pragma unroll
    for (int i = 0; i < D; ++i) w.d[i] = __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4 * i, soff, 0);
    if constexpr (NB % 4 >= 2) w.h = __builtin_amdgcn_raw_buffer_load_b16(r, voff + 4 * D, soff, 0);
    if constexpr (NB % 2 == 1) w.y = __builtin_amdgcn_raw_buffer_load_b8(r, voff + NB - 1, soff, 0);
}
template <int NB, int I>
__device__ __forceinline__ uint32_t byte_of(const RawRow<NB>& w)
{
    constexpr int D = NB / 4;  // whole dwords
    if constexpr (I < 4 * D) return (w.d[I / 4] >> (8 * (I % 4))) & 0xffu;
    else if constexpr (NB % 4 >= 2 && I < 4 * D + 2) return ((uint32_t)w.h >> (8 * (I - 4 * D))) & 0xffu;
    else return (uint32_t)w.y;
}

// byte_of with the index as an argument (constant after unrolling).
template <int NB>
__device__ __forceinline__ uint32_t byte_at(const RawRow<NB>& w, int i)
{
    constexpr int D = NB / 4;
    if (i < 4 * D) return (w.d[i / 4] >> (8 * (i % 4))) & 0xffu;
    if (NB % 4 >= 2 && i < 4 * D + 2) return ((uint32_t)w.h >> (8 * (i - 4 * D))) & 0xffu;
    return (uint32_t)w.y;
}

// Gray value of each of the lane's K columns from its packed input bytes.
template <int K, bool RGB, int... k>
__device__ __forceinline__ void gray_row(const RawRow<RowState<K, RGB>::NB>& w, float (&gr)[K],
                                         std::integer_sequence<int, k...>)
{
    constexpr int NB = RowState<K, RGB>::NB;
    if constexpr (RGB)
        ((gr[k] = (float)rgb2gray(byte_of<NB, 3 * k>(w), byte_of<NB, 3 * k + 1>(w), byte_of<NB, 3 * k + 2>(w))), ...);
    else
        ((gr[k] = (float)byte_of<NB, k>(w)), ...);
}

// The K*C input bytes of this lane in input row `row`, packed.  The row is
// clamped into the frame (a wavefront-uniform scalar operation), so the load
// can be issued on every row step, in range, whether or not the row is used:
// an unconditional load lets the compiler count the loads still in flight
// and wait only for the one a step needs, instead of for all of them at the
// join after a conditional load.  Every strip lies inside the frame.
template <int K, bool RGB>
__device__ __forceinline__ void load_raw(const RowCtx& c, int row, RawRow<RowState<K, RGB>::NB>& raw)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)c.in_frame, (short)0, c.row_bytes * c.Hf, 0x00020000);
    const int rc = row < 0 ? 0 : (row >= c.Hf ? c.Hf - 1 : row);
    load_words<RowState<K, RGB>::NB>(r, c.lane_in, rc * c.row_bytes, raw);
}

template <int K, bool RGB, bool DIFF, bool EL, bool ER, int U>
__device__ __forceinline__ void row_step(RowState<K, RGB>& st, const RowCtx& c, const SegParams& p, int j)
{
    constexpr int U3 = U % 3, U5 = U % 5;
    const int row_in = c.y0 - ROW_HX + j;

    // prefetch the input row two iterations ahead
    {
        const int rp = row_in + 2;
        load_raw<K, RGB>(c, rp, st.raw[(U + 2) % 3]);  // unused when rp is outside [lo_in, hi_in)
    }
    // Gaussian, horizontal pass, on the gray input row
    if ((unsigned)(j - c.ji) < (unsigned)c.ni) {
        float gr[K];
        gray_row<K, RGB>(st.raw[U3], gr, std::make_integer_sequence<int, K>{});
        float e[K + 4];
        extend_row<K, 2, EL, ER>(gr, e);
#pragma unroll
        for (int k = 0; k < K; ++k) st.h[U5][k] = gauss5_taps(p.gw, e[k], e[k + 1], e[k + 2], e[k + 3], e[k + 4]);
        if (row_in == 0) {
            copy_row<K>(st.h[(U + 4) % 5], st.h[U5]);
            copy_row<K>(st.h[(U + 3) % 5], st.h[U5]);
        }
    }
    // Gaussian, vertical pass: row row_in - 2
    const int rg = row_in - 2;
    if ((unsigned)(j - c.jg) < (unsigned)c.ng) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            st.g[U3][k] = gauss5_taps(p.gw, st.h[(U + 1) % 5][k], st.h[(U + 2) % 5][k], st.h[(U + 3) % 5][k],
                                      st.h[(U + 4) % 5][k], st.h[U5][k]);
        if (__builtin_expect(rg == 0, 0)) copy_row<K>(st.g[(U + 2) % 3], st.g[U3]);
    }
    // Sobel, products and the horizontal pass of the window sums: row row_in - 3
    const int rs = row_in - 3;
    float bn[3][K];  // horizontal pass of row rs
    if ((unsigned)(j - c.js) < (unsigned)c.ns) {
        float sv[K], ev[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float gm = st.g[(U + 1) % 3][k], g0 = st.g[(U + 2) % 3][k], gp = st.g[U3][k];
            sv[k] = sobel_sv(gm, g0, gp);
            ev[k] = sobel_e(gm, gp);
        }
        float esv[K + 2], eev[K + 2];
        extend_row<K, 1, EL, ER>(sv, esv);
        extend_row<K, 1, EL, ER>(ev, eev);
        float pr[3][K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float ix = sobel_ix(esv[k], esv[k + 2]);
            const float iy = sobel_iy(eev[k], eev[k + 1], eev[k + 2]);
            products(ix, iy, pr[0][k], pr[1][k], pr[2][k]);
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) box5_row<K, EL, ER>(pr[ch], bn[ch]);
        if (rs == 0) {  // the row above the frame's first row is that row
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) copy_row<K>(st.bp[ch], bn[ch]);
        }
    } else {
        // below the frame's last row: the replicate border (elsewhere unused)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) copy_row<K>(bn[ch], st.bp[ch]);
    }
    // Window sums (vertical), Harris, threshold, 3-wide maximum: row row_in - 5
    const int rb = row_in - 5;
    if ((unsigned)(j - c.jb) < (unsigned)c.nb) {
        // sum5 over rows rb-2 .. rb+2: (q_(rb-2) + q_rb) + b_(rb+2), the same
        // operations in the same order, with each row pair added once
        // (the pair of the two newest rows replaces q_(rb-2) right after its read)
        float s[3][K];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                s[ch][k] = (st.q[U3][ch][k] + st.q[(U + 2) % 3][ch][k]) + bn[ch][k];
                st.q[U3][ch][k] = st.bp[ch][k] + bn[ch][k];
            }
#pragma unroll
        for (int k = 0; k < K; ++k) st.rt[U3][k] = threshold(harris(s[0][k], s[1][k], s[2][k], p.k), p.thr);
        float e[K + 2];
        extend_row<K, 1, EL, ER>(st.rt[U3], e);
#pragma unroll
        for (int k = 0; k < K; ++k) st.m[U3][k] = max3(e[k], e[k + 1], e[k + 2]);
        if (rb == 0) {
            copy_row<K>(st.rt[(U + 2) % 3], st.rt[U3]);
            copy_row<K>(st.m[(U + 2) % 3], st.m[U3]);
        }
    }
    // Row pair q_(rs-1) = b_(rs-1) + b_rs on the iterations whose window sums
    // did not already form it (the first ones of the band); at the frame's
    // first row the two pairs above it are both twice row 0 (replicate border)
    if ((unsigned)(j - c.jq) < (unsigned)c.nq) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
            for (int k = 0; k < K; ++k) st.q[U3][ch][k] = st.bp[ch][k] + bn[ch][k];
        if (rs == 0) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) copy_row<K>(st.q[(U + 2) % 3][ch], st.q[U3][ch]);
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) copy_row<K>(st.bp[ch], bn[ch]);
    // Suppression, feature points, output: row row_in - 6
    const int rn = row_in - 6;
    if ((unsigned)(j - c.jn) < (unsigned)c.nn) {
        uint32_t bits = 0;
        float centre[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float wmax = max3(st.m[(U + 1) % 3][k], st.m[(U + 2) % 3][k], st.m[U3][k]);
            centre[k] = st.rt[(U + 2) % 3][k];
            bits |= (nms_keep(centre[k], wmax) != 0u ? 1u : 0u) << k;
        }
        const uint32_t pts = bits & c.valid;
        if (p.count != nullptr && c.real && __ballot(pts != 0u) != 0ull) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                emit_points(p, (pts >> k & 1u) != 0u, (uint32_t)c.t, (uint32_t)rn, (uint32_t)(c.x0 + K * c.lane + k),
                            centre[k]);
        }
        uint32_t outbits = bits;
        if constexpr (DIFF) {
            uint8_t* slot = c.prev + (rn - c.y0) * 64 + c.lane;
            const uint32_t prev = c.t == 0 ? bits : (uint32_t)*slot;
            *slot = (uint8_t)bits;
            outbits = bits ^ prev;
        }
        if (c.store) {
            const __amdgpu_buffer_rsrc_t r = out_rsrc(c.out_frame, (uint32_t)(c.W * c.Hf));
            const int soff = rn * c.W;  // uniform row offset
#pragma unroll
            for (int k = 0; k < K; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((outbits >> k & 1u) ? (uint8_t)255 : (uint8_t)0, r,
                                                     (c.valid >> k & 1u) ? c.lane_out + k : DROP, soff, 0);
        }
    }
    // bottom replicate of the Gaussian and response rings: after the last
    // frame row, copy it into the next slot, once per iteration, for as many
    // rows as the consumer reads (rare: branches, not selects on every row)
    if (__builtin_expect(row_in >= c.Hf - 1 && row_in <= c.Hf, 0)) copy_row<K>(st.h[(U + 1) % 5], st.h[U5]);
    if (__builtin_expect(rg == c.Hf - 1, 0)) copy_row<K>(st.g[(U + 1) % 3], st.g[U3]);
    if (rb == c.Hf - 1) {
        copy_row<K>(st.rt[(U + 1) % 3], st.rt[U3]);
        copy_row<K>(st.m[(U + 1) % 3], st.m[U3]);
    }
}

template <int K, bool RGB, bool DIFF, bool EL, bool ER, int... U>
__device__ __forceinline__ void row_block(RowState<K, RGB>& st, const RowCtx& c, const SegParams& p, int jb, int n,
                                          std::integer_sequence<int, U...>)
{
    ((jb + U < n ? row_step<K, RGB, DIFF, EL, ER, U>(st, c, p, jb + U) : void()), ...);
}

// One side of a frame boundary between two runs of frames of the same strip
// and band: the mask of the frame next to the boundary on this side (held in
// the LDS row of previous-frame bits) is published as K ballot words per row;
// the side that arrives second reads the other side's words and writes the
// frame difference of the later run's first frame (out_frame): the exclusive
// or of the two masks, the same bits the later item would have formed from a
// recomputed frame.  Neither side waits for the other.
//
// Every access to the exchange words and the counter is a device-scope
// atomic read-modify-write, which the device performs coherently across its
// XCDs; the words are published with exchanges whose results are waited for
// before the arrival is counted, and read (fetch-or 0) only after the count
// has come back.  No fence is used: an agent-scope release or acquire fence
// writes back or invalidates the XCD's whole L2, which cost the kernel a
// quarter of its speed (the strips of neighbouring items share input rows
// in L2).
template <int K>
__device__ __forceinline__ void row_exchange(const RowCtx& c, uint64_t* mine, uint64_t* other, uint32_t* cnt,
                                             uint8_t* out_frame)
{
    constexpr int RPC = 64 / K;  // rows per chunk: one word per lane
    const int nrow = c.y1 - c.y0;
    uint64_t sink = 0;
    for (int r0 = 0; r0 < nrow; r0 += RPC) {
        const int nr = min(RPC, nrow - r0);
        uint64_t w = 0;  // lane (r - r0) K + k: word k of row r
        for (int r = 0; r < nr; ++r) {
            const uint32_t b = c.prev[(r0 + r) * 64 + c.lane];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t m = __ballot((b >> k & 1u) != 0u);
                if (c.lane == r * K + k) w = m;
            }
        }
        if (c.lane < nr * K)
            sink |= __hip_atomic_exchange(mine + r0 * K + c.lane, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the exchanges have returned (so they are performed) before the arrival
    // is counted: the empty asm needs their results, and orders the memory
    // operations around it
    const uint32_t sl = (uint32_t)sink, sh = (uint32_t)(sink >> 32);
    asm volatile("" ::"v"(sl), "v"(sh) : "memory");
    uint32_t old = 0;
    if (c.lane == 0) old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __builtin_amdgcn_readfirstlane(__shfl(old, 0));
    if (old == 0u) return;
    const __amdgpu_buffer_rsrc_t rs = out_rsrc(out_frame, (uint32_t)(c.W * c.Hf));
    for (int r0 = 0; r0 < nrow; r0 += RPC) {
        const int nr = min(RPC, nrow - r0);
        uint64_t w = 0;
        if (c.lane < nr * K)
            w = __hip_atomic_fetch_or(other + r0 * K + c.lane, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int r = 0; r < nr; ++r) {
            const uint32_t b = c.prev[(r0 + r) * 64 + c.lane];
            uint32_t o = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t m = __shfl(w, r * K + k);
                o |= (uint32_t)(m >> c.lane & 1u) << k;
            }
            const uint32_t outbits = b ^ o;
            const int soff = (c.y0 + r0 + r) * c.W;
#pragma unroll
            for (int k = 0; k < K; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((outbits >> k & 1u) ? (uint8_t)255 : (uint8_t)0, rs,
                                                     (c.valid >> k & 1u) ? c.lane_out + k : DROP, soff, 0);
        }
    }
}

// Exchange areas of the boundary before run `chunk` (chunk >= 1).
struct RowBoundary {
    uint64_t* last;   // the earlier run's last frame
    uint64_t* first;  // the later run's first frame
    uint32_t* cnt;
};
template <int K>
__device__ __forceinline__ RowBoundary row_boundary(const RowParams& rp, int strip, int band, int chunk)
{
    const size_t b = ((size_t)(chunk - 1) * rp.nbands + band) * rp.nstrips + strip;
    const size_t words = (size_t)rp.band_h * K;
    return RowBoundary{rp.xmask + 2 * b * words, rp.xmask + (2 * b + 1) * words, rp.xcount + b};
}

// All frames of one work item.
template <int K, bool RGB, bool DIFF, bool EL, bool ER>
__device__ __forceinline__ void row_frames(RowCtx& c, const RowParams& rp, int strip, int band, int ts, int t0,
                                           int t1)
{
    const SegParams& p = rp.sp;
    constexpr int C = RGB ? 3 : 1;
    const size_t plane = (size_t)p.W * p.H;
    const int n = c.y1 - c.y0 + 2 * ROW_HX;
    const bool xch = DIFF && rp.xcount != nullptr;
    for (int t = ts; t < t1; ++t) {
        c.t = t;
        c.real = t >= t0;
        c.store = c.real && !(xch && t == t0 && t0 > 0);
        c.in_frame = (const uint8_t*)p.in + (size_t)t * plane * C;
        c.out_frame = (uint8_t*)p.out + (size_t)t * plane;
        RowState<K, RGB> st;
        // first two input rows
        const int r0 = c.y0 - ROW_HX;
        load_raw<K, RGB>(c, r0, st.raw[0]);
        load_raw<K, RGB>(c, r0 + 1, st.raw[1]);
        for (int jb = 0; jb < n; jb += ROW_UNROLL)
            row_block<K, RGB, DIFF, EL, ER>(st, c, p, jb, n, std::make_integer_sequence<int, ROW_UNROLL>{});
        if constexpr (DIFF) {
            if (xch && t == t0 && t0 > 0) {  // the boundary before the run: this side is its first frame
                const RowBoundary x = row_boundary<K>(rp, strip, band, t0 / rp.tt);
                row_exchange<K>(c, x.first, x.last, x.cnt, c.out_frame);
            }
            if (xch && t == t1 - 1 && t1 < p.T) {  // the boundary after the run: this side is its last frame
                const RowBoundary x = row_boundary<K>(rp, strip, band, t1 / rp.tt);
                row_exchange<K>(c, x.last, x.first, x.cnt, (uint8_t*)p.out + (size_t)t1 * plane);
            }
        }
    }
}

// Geometry of one work item: strip, band and frame run of one clip.
struct RowItem {
    int strip, band, chunk;
    int nstrips, band_h, tt, strip_step;
};

// One work item of one wavefront (all of it wavefront-uniform).
template <int K, bool RGB, bool DIFF>
__device__ __forceinline__ void row_item(const RowParams& rp, const RowItem& it, uint8_t* prev_lds)
{
    const SegParams& p = rp.sp;
    RowCtx c;
    c.W = p.W;
    c.Hf = p.H;
    c.lane = threadIdx.x & 63;
    const int S = it.strip_step;
    c.x0 = min(it.strip * S, p.W - 64 * K);
    constexpr int CIN = RGB ? 3 : 1;
    c.row_bytes = p.W * CIN;
    c.lane_in = (c.x0 + K * c.lane) * CIN;
    c.lane_out = c.x0 + K * c.lane;
    const int vx0 = it.strip == 0 ? 0 : (it.strip - 1) * S + 64 * K - ROW_HX;
    const int vx1 = it.strip == it.nstrips - 1 ? p.W : it.strip * S + 64 * K - ROW_HX;
    c.valid = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int x = c.x0 + K * c.lane + k;
        c.valid |= (x >= vx0 && x < vx1 ? 1u : 0u) << k;
    }
    c.y0 = it.band * it.band_h;
    c.y1 = min(c.y0 + it.band_h, p.H);
    c.lo_in = max(0, c.y0 - 6);
    c.hi_in = min(p.H, c.y1 + 6);
    c.lo_g = max(0, c.y0 - 4);
    c.hi_g = min(p.H, c.y1 + 4);
    c.lo_s = max(0, c.y0 - 3);
    c.hi_s = min(p.H, c.y1 + 3);
    c.lo_b = max(0, c.y0 - 1);
    c.hi_b = min(p.H, c.y1 + 1);
    // row r of a stage with lag L (rows behind the input row) is computed at
    // iteration j = r - y0 + 6 + L
    const int base = ROW_HX - c.y0;
    c.jp = c.lo_in + base - 2;  // prefetch of row j + 2
    c.np_ = c.hi_in - c.lo_in;
    c.ji = c.lo_in + base;
    c.ni = c.hi_in - c.lo_in;
    c.jg = c.lo_g + base + 2;
    c.ng = c.hi_g - c.lo_g;
    c.js = c.lo_s + base + 3;
    c.ns = c.hi_s - c.lo_s;
    c.jb = c.lo_b + base + 5;
    c.nb = c.hi_b - c.lo_b;
    // row pairs q_(s-1): the window sums of rows [lo_b, hi_b) read q_(lo_b-2) ..
    // q_(hi_b-1), formed on the iterations s = max(lo_b - 1, lo_s) .. hi_b; from
    // s = lo_b + 2 on, the window-sum step forms them, so the pair step runs on
    // the iterations before it
    const int lo_q = max(c.lo_b - 1, c.lo_s);
    c.jq = lo_q + base + 3;
    c.nq = c.lo_b + 2 - lo_q;
    c.jn = c.y0 + base + 6;
    c.nn = c.y1 - c.y0;
    c.prev = prev_lds;

    const int t0 = it.chunk * it.tt;
    const int t1 = min(t0 + it.tt, p.T);
    const int ts = (DIFF && t0 > 0 && rp.xcount == nullptr) ? t0 - 1 : t0;
    const bool el = it.strip == 0, er = it.strip == it.nstrips - 1;
    if (el && er)
        row_frames<K, RGB, DIFF, true, true>(c, rp, it.strip, it.band, ts, t0, t1);
    else if (el)
        row_frames<K, RGB, DIFF, true, false>(c, rp, it.strip, it.band, ts, t0, t1);
    else if (er)
        row_frames<K, RGB, DIFF, false, true>(c, rp, it.strip, it.band, ts, t0, t1);
    else
        row_frames<K, RGB, DIFF, false, false>(c, rp, it.strip, it.band, ts, t0, t1);
}

// Decompose a clip-local item index.  Strips vary fastest, then bands, then
// frame runs: the wavefronts in flight cover whole frames, neighbouring
// wavefronts reading neighbouring segments of the same rows.  (With strips
// varying slowest, the wavefronts in flight covered one 128-column strip of
// hundreds of frames, and the memory-bound kernels ran at a third of the
// bandwidth.)
__device__ __forceinline__ RowItem row_decompose(int item, int nstrips, int nbands, int nchunks, int band_h, int tt,
                                                 int strip_step)
{
    RowItem it;
    it.strip = item % nstrips;
    const int rest = item / nstrips;
    it.band = rest % nbands;
    it.chunk = rest / nbands;
    it.nstrips = nstrips;
    it.band_h = band_h;
    it.tt = tt;
    it.strip_step = strip_step;
    return it;
}

template <int K, bool RGB, bool DIFF>
__global__ __launch_bounds__(ROW_WAVES * 64) void k_rowfuse(RowParams rp)
{
    extern __shared__ uint8_t row_lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
    const int item = blockIdx.x * ROW_WAVES + wave;
    if (item >= rp.total) return;  // whole wavefront leaves; no barrier is used
    const RowItem it = row_decompose(item, rp.nstrips, rp.nbands, rp.nchunks, rp.band_h, rp.tt, rp.strip_step);
    row_item<K, RGB, DIFF>(rp, it, row_lds + wave * rp.band_h * 64);
}

// ---------------------------------------------------------------- batches
// Many clips of different sizes in one persistent launch: every wavefront
// takes work items (clip, strip, band, frame run) from a queue counter until
// none are left.  Clip descriptors travel by value in the kernel arguments.
constexpr int FZ_BATCH_MAX = 32;
constexpr int BATCH_BAND_H = 64;
constexpr int BATCH_TT = 16;

struct BatchClip {
    const void* in;
    void* out;
    fz_point* points;
    uint32_t* count;
    int W, H, T;
    uint32_t cap;
    int nstrips, nbands, nchunks, item_begin;
};

struct BatchParams {
    Gauss5W gw;
    float k, thr;
    int n_clips, total;
    uint32_t* queue;  // work counter, zero at launch
    BatchClip clip[FZ_BATCH_MAX];
};

template <int K, bool RGB, bool DIFF>
__global__ __launch_bounds__(ROW_WAVES * 64) void k_rowfuse_batch(BatchParams bp)
{
    extern __shared__ uint8_t row_lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t v = 0;
        if (lane == 0) v = atomicAdd(bp.queue, 1u);
        const int item = __builtin_amdgcn_readfirstlane(__shfl(v, 0));
        if (item >= bp.total) break;  // every wave ends once the queue is drained
        int ci = 0;
        while (ci + 1 < bp.n_clips && item >= bp.clip[ci + 1].item_begin) ++ci;
        const BatchClip& bc = bp.clip[ci];
        RowParams rp{};
        SegParams& sp = rp.sp;
        sp.in = bc.in;
        sp.out = bc.out;
        sp.W = bc.W;
        sp.H = bc.H;
        sp.T = bc.T;
        sp.tpb = BATCH_TT;
        sp.gw = bp.gw;
        sp.k = bp.k;
        sp.thr = bp.thr;
        sp.points = bc.points;
        sp.count = bc.count;
        sp.cap = bc.cap;
        const RowItem it = row_decompose(item - bc.item_begin, bc.nstrips, bc.nbands, bc.nchunks, BATCH_BAND_H,
                                         BATCH_TT, 64 * K - 2 * ROW_HX);
        rp.tt = BATCH_TT;  // no exchange buffers: each run recomputes the frame before it
        row_item<K, RGB, DIFF>(rp, it, row_lds + wave * BATCH_BAND_H * 64);
    }
}

hipError_t launch_rowfuse_batch(const BatchParams& bp, int K, bool rgb, bool diff, int blocks, hipStream_t s);
int rowfuse_batch_blocks_per_cu(int K, bool rgb, bool diff);

hipError_t launch_rowfuse(const RowParams& rp, int K, bool rgb, bool diff, hipStream_t s);

}  // namespace fz
