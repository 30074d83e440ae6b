// Row-marching kernel for any contiguous group with a window stage of the
// compiled chains (Harris chain with or without the gray conversion, gradient
// chain), including single window stages.
//
// Organisation (see rowfuse.h for the same scheme written out for the whole
// Harris chain): a wavefront owns a strip of 64*K columns of a band of rows and
// marches down the rows.  Iteration j loads input row y0 - H + j (H = the
// group's halo) and every window stage S, in order,
//   * pushes the row it receives this iteration into its ring of 2r+1 rows
//     (Gaussian and window sums store their horizontal pass, the Sobel stage
//     its input, suppression its input and its 3-wide maximum), writing the
//     frame's first row also into the slots of the rows above it;
//   * emits its output row (vertical pass) when that row is needed by the
//     band, after which the point stages up to the next window stage run on it
//     in registers and the row goes to the next window stage;
//   * at the end of the iteration copies the frame's last row into the slots
//     below it, one slot per iteration.
// The last window stage's row, after the trailing point stages (and the frame
// difference through LDS mask bits), is stored.  Horizontal neighbours come
// through DPP wave shifts; at a frame edge the edge lane keeps its own value
// (replicate border).  Rings are fixed registers: the row loop is unrolled by
// 15 = lcm(3, 5).
#pragma once

#include "engine.h"
#include "rowfuse.h"

namespace fz {

template <int CH, int A, int B>
struct GenInfo {
    static constexpr bool DIFF = chain_op(CH, B) == FZ_OP_FRAMEDIFF;
    static constexpr int BL = DIFF ? B - 1 : B;  // last stage evaluated per row
    static constexpr int H = group_halo(CH, A, B);
    static constexpr OpInfo IN = op_info(chain_op(CH, A));
    static constexpr bool IN_RGB = IN.op == FZ_OP_RGB2GRAY;
    static constexpr bool IN_U8 = IN.in_dt == FZ_U8;
    static constexpr int IN_PLANES = IN_U8 ? 1 : IN.in_ch;         // f32 planes
    static constexpr int IN_BYTES = IN_RGB ? 3 : 1;                // bytes per pixel of a u8 input
    static constexpr int W0 = next_window(CH, A, BL);
    static constexpr int LASTW = [] {
        int w = -1;
        for (int j = A; j <= BL; ++j)
            if (is_window(CH, j)) w = j;
        return w;
    }();
    static constexpr bool has(int op)
    {
        for (int j = A; j <= BL; ++j)
            if (chain_op(CH, j) == op) return true;
        return false;
    }
    static constexpr bool HAS_NMS = has(FZ_OP_NMS3);
    // rows of lag before stage s's input: radii of the window stages before s
    static constexpr int lag_in(int s) { return H - halo_after(CH, s - 1, B); }
    static constexpr OpInfo OUT = op_info(chain_op(CH, B));
    static constexpr int OUT_CH = channels_after_step(CH, LASTW, BL);
};

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int CH, int A, int B, int K>
struct GenState {
    using I = GenInfo<CH, A, B>;
    float gh[I::has(FZ_OP_GAUSS5) ? 5 : 1][K];
    float sg[I::has(FZ_OP_SOBEL3) ? 3 : 1][K];
    float bh[I::has(FZ_OP_BOXSUM5) ? 5 : 1][3][K];
    float nr[I::HAS_NMS ? 3 : 1][K];
    float nm[I::HAS_NMS ? 3 : 1][K];
    // input rows, two loaded ahead: u8 bytes as loaded, or f32 words
    struct Raw {
        RawRow<I::IN_U8 ? K * I::IN_BYTES : 1> b;
        uint32_t f[I::IN_U8 ? 1 : K * I::IN_PLANES];
    } raw[3];
};

struct GenCtx {
    const void* in;
    void* out;
    int W, Hf, x0, lane, y0, y1, t;
    size_t plane, vol;  // pixels per frame, pixels per channel volume
    bool real;
    uint32_t valid;
    int lane_in;        // element offset of this lane's first column in an input row
    uint8_t* prev;
};

template <int K, int R, bool EDGE>
__device__ __forceinline__ void gen_extend(const float (&v)[K], float (&e)[K + 2 * R])
{
    extend_row<K, R, EDGE, EDGE>(v, e);
}

template <int CH, int A, int B, int K, class Raw>
__device__ __forceinline__ void gen_load(const GenCtx& c, int row, Raw& raw)
{
    using I = GenInfo<CH, A, B>;
    // buffers over frame t (of each plane), uniform row offset, lane offset;
    // the row is clamped into the frame so the load can be issued on every
    // step (see load_raw)
    row = row < 0 ? 0 : (row >= c.Hf ? c.Hf - 1 : row);
    const size_t fbase = (size_t)c.t * c.plane;
    if constexpr (I::IN_U8) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)((const uint8_t*)c.in + fbase * I::IN_BYTES), (short)0, (int)(c.plane * I::IN_BYTES), 0x00020000);
        load_words<K * I::IN_BYTES>(r, c.lane_in * I::IN_BYTES, row * c.W * I::IN_BYTES, raw.b);
    } else {
#pragma unroll
        for (int ch = 0; ch < I::IN_PLANES; ++ch) {
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                (void*)((const float*)c.in + ch * c.vol + fbase), (short)0, (int)(c.plane * 4), 0x00020000);
            const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, 4 * c.lane_in, 4 * row * c.W, 0);  // K == 2
            raw.f[ch * K] = w.x;
            raw.f[ch * K + 1] = w.y;
        }
    }
}

// Input row (after the group's leading point stages) as v[ch][k].
template <int CH, int A, int B, int K, class Raw>
__device__ __forceinline__ void gen_unpack(const Raw& raw, float (&v)[3][K], const SegParams& p)
{
    using I = GenInfo<CH, A, B>;
    constexpr int NB = K * I::IN_BYTES;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float px[3];
        if constexpr (I::IN_RGB) {
            px[0] = (float)byte_at<NB>(raw.b, 3 * k);
            px[1] = (float)byte_at<NB>(raw.b, 3 * k + 1);
            px[2] = (float)byte_at<NB>(raw.b, 3 * k + 2);
        } else if constexpr (I::IN_U8) {
            px[0] = (float)byte_at<NB>(raw.b, k);
        } else {
#pragma unroll
            for (int ch = 0; ch < I::IN_PLANES; ++ch) px[ch] = __uint_as_float(raw.f[ch * K + k]);
        }
        point_run<CH, A, pw_end(CH, A, B)>(px, p);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) v[ch][k] = px[ch];
    }
}

template <int K, class Fn>
__device__ __forceinline__ void apply_points_row(float (&v)[3][K], Fn&& f)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float px[3] = {v[0][k], v[1][k], v[2][k]};
        f(px);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) v[ch][k] = px[ch];
    }
}

// Store the final row (or its frame difference) for the valid columns; the
// other lanes' stores get an out-of-range offset and are dropped.
template <int CH, int A, int B, int K>
__device__ __forceinline__ void gen_store(const GenCtx& c, int row, const float (&v)[3][K], uint32_t outbits)
{
    using I = GenInfo<CH, A, B>;
    const size_t fbase = (size_t)c.t * c.plane;
    const int soff = row * c.W;  // uniform row offset (elements)
    // With two columns per lane, a lane that owns both writes them with one
    // access (a contiguous segment per wavefront instead of two interleaved
    // half-filled ones); the few lanes at a strip boundary that own one
    // column write it alone.  Dropped (out-of-range) offsets do the masking.
    static_assert(K == 2, "the generic row kernel runs two columns per lane");
    const bool both = c.valid == 3u;
    const int lo = (!both && (c.valid & 1u)) ? c.lane_in : DROP;
    const int hi = (!both && (c.valid & 2u)) ? c.lane_in + 1 : DROP;
    if constexpr (I::DIFF || I::OUT.out_dt == FZ_U8) {
        const __amdgpu_buffer_rsrc_t r = out_rsrc((uint8_t*)c.out + fbase, (uint32_t)c.plane);
        uint32_t b[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (I::DIFF || I::OUT.op == FZ_OP_NMS3)
                b[k] = (outbits >> k & 1u) ? 255u : 0u;
            else
                b[k] = (uint32_t)v[0][k];
        }
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(b[0] | b[1] << 8), r, both ? c.lane_in : DROP, soff, 0);
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)b[0], r, lo, soff, 0);
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)b[1], r, hi, soff, 0);
    } else {
#pragma unroll
        for (int ch = 0; ch < I::OUT_CH; ++ch) {
            const __amdgpu_buffer_rsrc_t r = out_rsrc((float*)c.out + ch * c.vol + fbase, (uint32_t)(c.plane * 4));
            u32x2 w;
            w.x = __float_as_uint(v[ch][0]);
            w.y = __float_as_uint(v[ch][1]);
            __builtin_amdgcn_raw_buffer_store_b64(w, r, both ? 4 * c.lane_in : DROP, 4 * soff, 0);
            __builtin_amdgcn_raw_buffer_store_b32(w.x, r, lo == DROP ? DROP : 4 * lo, 4 * soff, 0);
            __builtin_amdgcn_raw_buffer_store_b32(w.y, r, hi == DROP ? DROP : 4 * hi, 4 * soff, 0);
        }
    }
}

template <int CH, int A, int B, int K, bool EDGE, int S, int U>
__device__ __forceinline__ void gen_window(GenState<CH, A, B, K>& st, const GenCtx& c, const SegParams& p, int r_in,
                                           bool have, float (&v)[3][K]);

// Window stages from S on (S > last window: the final row, stored).
template <int CH, int A, int B, int K, bool EDGE, int S, int U>
__device__ __forceinline__ void gen_from(GenState<CH, A, B, K>& st, const GenCtx& c, const SegParams& p, int r_in,
                                         bool have, float (&v)[3][K])
{
    using I = GenInfo<CH, A, B>;
    if constexpr (S <= I::LASTW) {
        gen_window<CH, A, B, K, EDGE, S, U>(st, c, p, r_in, have, v);
    } else {
        // r_in is the final row; `have` says it was produced and lies in the band
        if (have) {
            uint32_t bits = 0;
            if constexpr (I::HAS_NMS) {
#pragma unroll
                for (int k = 0; k < K; ++k) bits |= ((uint32_t)v[0][k] != 0u ? 1u : 0u) << k;
                const uint32_t pts = bits & c.valid;
                if (p.count != nullptr && c.real && __ballot(pts != 0u) != 0ull) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        emit_points(p, (pts >> k & 1u) != 0u, (uint32_t)c.t, (uint32_t)r_in,
                                    (uint32_t)(c.lane_in + k), v[1][k]);
                }
            }
            uint32_t outbits = bits;
            if constexpr (I::DIFF) {
                uint8_t* slot = c.prev + (r_in - c.y0) * 64 + c.lane;
                const uint32_t prev = c.t == 0 ? bits : (uint32_t)*slot;
                *slot = (uint8_t)bits;
                outbits = bits ^ prev;
            }
            if (c.real) gen_store<CH, A, B, K>(c, r_in, v, outbits);
        }
    }
}

template <int CH, int A, int B, int K, bool EDGE, int S, int U>
__device__ __forceinline__ void gen_window(GenState<CH, A, B, K>& st, const GenCtx& c, const SegParams& p, int r_in,
                                           bool have, float (&v)[3][K])
{
    using I = GenInfo<CH, A, B>;
    constexpr int OP = chain_op(CH, S);
    constexpr int R = op_info(OP).r;
    constexpr int hout = halo_after(CH, S, B);
    constexpr int NXT = next_window(CH, S + 1, I::BL);
    constexpr int E = pw_end(CH, S + 1, B);
    constexpr int U3 = U % 3, U5 = U % 5;
    const int r_out = r_in - R;
    const int lo = max(0, c.y0 - hout), hi = min(c.Hf, c.y1 + hout);
    const bool emit = r_out >= lo && r_out < hi;
    float o[3][K];

    if constexpr (OP == FZ_OP_GAUSS5) {
        if (have) {
            float e[K + 4];
            float row[K];
#pragma unroll
            for (int k = 0; k < K; ++k) row[k] = v[0][k];
            gen_extend<K, 2, EDGE>(row, e);
#pragma unroll
            for (int k = 0; k < K; ++k) st.gh[U5][k] = gauss5_taps(p.gw, e[k], e[k + 1], e[k + 2], e[k + 3], e[k + 4]);
            if (r_in == 0) {
                copy_row<K>(st.gh[(U + 4) % 5], st.gh[U5]);
                copy_row<K>(st.gh[(U + 3) % 5], st.gh[U5]);
            }
        }
        if (emit) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                o[0][k] = gauss5_taps(p.gw, st.gh[(U + 1) % 5][k], st.gh[(U + 2) % 5][k], st.gh[(U + 3) % 5][k],
                                      st.gh[(U + 4) % 5][k], st.gh[U5][k]);
        }
    } else if constexpr (OP == FZ_OP_SOBEL3) {
        if (have) {
#pragma unroll
            for (int k = 0; k < K; ++k) st.sg[U3][k] = v[0][k];
            if (r_in == 0) copy_row<K>(st.sg[(U + 2) % 3], st.sg[U3]);
        }
        if (emit) {
            float sv[K], ev[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float gm = st.sg[(U + 1) % 3][k], g0 = st.sg[(U + 2) % 3][k], gp = st.sg[U3][k];
                sv[k] = sobel_sv(gm, g0, gp);
                ev[k] = sobel_e(gm, gp);
            }
            float esv[K + 2], eev[K + 2];
            gen_extend<K, 1, EDGE>(sv, esv);
            gen_extend<K, 1, EDGE>(ev, eev);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                o[0][k] = sobel_ix(esv[k], esv[k + 2]);
                o[1][k] = sobel_iy(eev[k], eev[k + 1], eev[k + 2]);
            }
        }
    } else if constexpr (OP == FZ_OP_BOXSUM5) {
        if (have) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float e[K + 4];
                float row[K];
#pragma unroll
                for (int k = 0; k < K; ++k) row[k] = v[ch][k];
                gen_extend<K, 2, EDGE>(row, e);
#pragma unroll
                for (int k = 0; k < K; ++k) st.bh[U5][ch][k] = sum5(e[k], e[k + 1], e[k + 2], e[k + 3], e[k + 4]);
            }
            if (r_in == 0) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    copy_row<K>(st.bh[(U + 4) % 5][ch], st.bh[U5][ch]);
                    copy_row<K>(st.bh[(U + 3) % 5][ch], st.bh[U5][ch]);
                }
            }
        }
        if (emit) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
#pragma unroll
                for (int k = 0; k < K; ++k)
                    o[ch][k] = sum5(st.bh[(U + 1) % 5][ch][k], st.bh[(U + 2) % 5][ch][k], st.bh[(U + 3) % 5][ch][k],
                                    st.bh[(U + 4) % 5][ch][k], st.bh[U5][ch][k]);
        }
    } else {
        static_assert(OP == FZ_OP_NMS3, "window stage");
        static_assert(hout == 0, "suppression must be the group's last window stage");
        if (have) {
            float row[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                row[k] = v[0][k];
                st.nr[U3][k] = row[k];
            }
            float e[K + 2];
            gen_extend<K, 1, EDGE>(row, e);
#pragma unroll
            for (int k = 0; k < K; ++k) st.nm[U3][k] = max3(e[k], e[k + 1], e[k + 2]);
            if (r_in == 0) {
                copy_row<K>(st.nr[(U + 2) % 3], st.nr[U3]);
                copy_row<K>(st.nm[(U + 2) % 3], st.nm[U3]);
            }
        }
        if (emit) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float wmax = max3(st.nm[(U + 1) % 3][k], st.nm[(U + 2) % 3][k], st.nm[U3][k]);
                const float centre = st.nr[(U + 2) % 3][k];
                o[0][k] = (float)nms_keep(centre, wmax);
                o[1][k] = centre;
            }
        }
    }
    if (emit) apply_points_row<K>(o, [&](float* px) { point_run<CH, S + 1, E>(px, p); });
    gen_from<CH, A, B, K, EDGE, NXT, U>(st, c, p, r_out, emit, o);

    // bottom replicate of this stage's ring, after every reader of this iteration
    if (r_in >= c.Hf - 1 && r_in <= c.Hf + R - 2) {
        if constexpr (OP == FZ_OP_GAUSS5) copy_row<K>(st.gh[(U + 1) % 5], st.gh[U5]);
        if constexpr (OP == FZ_OP_SOBEL3) copy_row<K>(st.sg[(U + 1) % 3], st.sg[U3]);
        if constexpr (OP == FZ_OP_BOXSUM5) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) copy_row<K>(st.bh[(U + 1) % 5][ch], st.bh[U5][ch]);
        }
        if constexpr (OP == FZ_OP_NMS3) {
            copy_row<K>(st.nr[(U + 1) % 3], st.nr[U3]);
            copy_row<K>(st.nm[(U + 1) % 3], st.nm[U3]);
        }
    }
}

template <int CH, int A, int B, int K, bool EDGE, int U>
__device__ __forceinline__ void gen_step(GenState<CH, A, B, K>& st, const GenCtx& c, const SegParams& p, int j)
{
    using I = GenInfo<CH, A, B>;
    const int row_in = c.y0 - I::H + j;
    const int lo_in = max(0, c.y0 - I::H), hi_in = min(c.Hf, c.y1 + I::H);
    const int rp = row_in + 2;
    gen_load<CH, A, B, K>(c, rp, st.raw[(U + 2) % 3]);  // unused when rp is outside [lo_in, hi_in)
    const bool have = row_in >= lo_in && row_in < hi_in;
    float v[3][K];
    if (have) gen_unpack<CH, A, B, K>(st.raw[U % 3], v, p);
    gen_from<CH, A, B, K, EDGE, I::W0, U>(st, c, p, row_in, have, v);
}

template <int CH, int A, int B, int K, bool EDGE, int... U>
__device__ __forceinline__ void gen_block(GenState<CH, A, B, K>& st, const GenCtx& c, const SegParams& p, int jb,
                                          int n, std::integer_sequence<int, U...>)
{
    ((jb + U < n ? gen_step<CH, A, B, K, EDGE, U>(st, c, p, jb + U) : void()), ...);
}

template <int CH, int A, int B, int K, bool EDGE>
__device__ __forceinline__ void gen_frames(GenCtx& c, const SegParams& p, int ts, int t0, int t1)
{
    using I = GenInfo<CH, A, B>;
    const int n = c.y1 - c.y0 + 2 * I::H;
    const int lo_in = max(0, c.y0 - I::H), hi_in = min(c.Hf, c.y1 + I::H);
    for (int t = ts; t < t1; ++t) {
        c.t = t;
        c.real = t >= t0;
        GenState<CH, A, B, K> st;
        const int r0 = c.y0 - I::H;
        gen_load<CH, A, B, K>(c, r0, st.raw[0]);
        gen_load<CH, A, B, K>(c, r0 + 1, st.raw[1]);
        for (int jb = 0; jb < n; jb += ROW_UNROLL)
            gen_block<CH, A, B, K, EDGE>(st, c, p, jb, n, std::make_integer_sequence<int, ROW_UNROLL>{});
    }
}

template <int CH, int A, int B, int K>
__device__ __forceinline__ void gen_item(const SegParams& p, const RowItem& it, uint8_t* prev_lds)
{
    using I = GenInfo<CH, A, B>;
    GenCtx c;
    c.in = p.in;
    c.out = p.out;
    c.W = p.W;
    c.Hf = p.H;
    c.plane = (size_t)p.W * p.H;
    c.vol = c.plane * p.T;
    c.lane = threadIdx.x & 63;
    const int S = it.strip_step;
    const int x0 = min(it.strip * S, p.W - 64 * K);
    c.x0 = x0;
    c.lane_in = x0 + K * c.lane;
    const int vx0 = it.strip == 0 ? 0 : (it.strip - 1) * S + 64 * K - I::H;
    const int vx1 = it.strip == it.nstrips - 1 ? p.W : it.strip * S + 64 * K - I::H;
    c.valid = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int x = c.lane_in + k;
        c.valid |= (x >= vx0 && x < vx1 ? 1u : 0u) << k;
    }
    c.y0 = it.band * it.band_h;
    c.y1 = min(c.y0 + it.band_h, p.H);
    c.prev = prev_lds;
    const int t0 = it.chunk * it.tt;
    const int t1 = min(t0 + it.tt, p.T);
    const int ts = (I::DIFF && t0 > 0) ? t0 - 1 : t0;
    if (it.strip == 0 || it.strip == it.nstrips - 1)
        gen_frames<CH, A, B, K, true>(c, p, ts, t0, t1);
    else
        gen_frames<CH, A, B, K, false>(c, p, ts, t0, t1);
}

template <int CH, int A, int B, int K>
__global__ __launch_bounds__(ROW_WAVES * 64) void k_rowgen(RowParams rp)
{
    extern __shared__ uint8_t gen_lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = blockIdx.x * ROW_WAVES + wave;
    if (item >= rp.total) return;
    const RowItem it = row_decompose(item, rp.nstrips, rp.nbands, rp.nchunks, rp.band_h, rp.tt, rp.strip_step);
    gen_item<CH, A, B, K>(rp.sp, it, gen_lds + wave * rp.band_h * 64);
}

template <int CH, int A, int B, int K>
hipError_t launch_rowgen_t(const RowParams& rp, hipStream_t s)
{
    if constexpr (A > B || B >= chain_len(CH) || !group_has_window(CH, A, B)) {
        return hipErrorInvalidValue;
    } else {
        const int blocks = (rp.total + ROW_WAVES - 1) / ROW_WAVES;
        const size_t lds = GenInfo<CH, A, B>::DIFF ? (size_t)ROW_WAVES * rp.band_h * 64 : 0;
        hipLaunchKernelGGL((k_rowgen<CH, A, B, K>), dim3(blocks), dim3(ROW_WAVES * 64), lds, s, rp);
        return hipGetLastError();
    }
}

using RowGenFn = hipError_t (*)(const RowParams&, hipStream_t);

}  // namespace fz
