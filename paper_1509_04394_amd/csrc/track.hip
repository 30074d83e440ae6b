// Kalman tracking of the extracted feature points: the stage after the chain.
//
// The paper's pipeline ends by applying a Kalman filter to the feature points
// (Sec. III; Table II: a single-point, multi-frame operation); Table IV marks
// it kernel-to-kernel dependent, so it is never fused with the kernels before
// it and runs here as its own launches on the chain's point list.  The model
// (the paper gives none) is the discrete Kalman filter with a constant-
// velocity state s = (x, y, vx, vy):
//   F = [[1,0,1,0],[0,1,0,1],[0,0,1,0],[0,0,0,1]],
//   Q = q [[1/4,0,1/2,0],[0,1/4,0,1/2],[1/2,0,1,0],[0,1/2,0,1]],
//   H = [[1,0,0,0],[0,1,0,0]], R = r I,
// with greedy nearest-neighbour association by Mahalanobis distance d2 =
// nu^T S^-1 nu (candidates d2 <= gate, taken in increasing (d2, track id,
// point index) order), a track dropped after more than max_miss missed frames
// in a row, and a new track, s = (x, y, 0, 0), P = diag(r, r, v0, v0), for
// every point left over (ids in (y, x) order).  All arithmetic is double
// precision, every matrix product the plain sum over k = 0, 1, ... from 0.0,
// evaluated without contraction: the association is a discrete decision, and
// this makes it (and every state) reproducible to the bit.  Products with F
// and H (entries 0 and 1) are written out term by term; they give the same
// bits as those sums (see f_row).
//
// Launches: the points are bucketed by frame (a histogram, one scan, a
// scatter into the workspace), then one workgroup marches the frames in
// order: it sorts the frame's points by (y, x) (rank by counting), predicts
// every live track, lists the gated candidate pairs and takes them greedily
// in rounds of candidates that come first for both their track and their
// point (no sort of the candidates), updates the tracks, appends the new
// ones and writes one record per live track.  The list is kept in id order: its first
// 64 tracks in registers, the rest in the workspace in two buffers
// (ping-pong on compaction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "fz_internal.h"

namespace fz {

constexpr int TRK_THREADS = 64;       // lanes of a wavefront: the tracks of the list it keeps in registers
constexpr int TRK_WAVES = 4;          // wavefronts that march the frames together
constexpr int TRK_GROUP = 5;          // points a wavefront tests at a time in the candidate search
constexpr int TRK_ASSOC_REG = 2;      // candidates per lane the association keeps in registers
constexpr int TRK_MAX_POINTS = 1024;  // points of one frame
constexpr int TRK_MAX_CANDS = 2048;   // gated (track, point) pairs of one frame

struct DevTrack {
    int32_t id, miss;
    int32_t status, pad;  // 0 predicted only, 1 updated, 2 started (this frame)
    double s[4];
    double P[16];
    double Si[4];  // S^-1 of the current frame's prediction
};

struct TrkState {  // workspace header
    uint32_t n_tracks, next_id, cur;
    uint32_t pad;
};

// C = A (n x m) B (m x p), row-major, plain sums from 0.0 in k order
template <int N, int M, int P>
__device__ __forceinline__ void mm(const double* A, const double* B, double* C)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < P; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) acc = acc + A[i * M + k] * B[k * P + j];
            C[i * P + j] = acc;
        }
}

// Products with F, H and their transposes, written out.  Their entries are
// 0 and 1, so every term of the plain sum (from 0.0, in k order) is exact: a
// copy of an operand, or a zero.  A partial sum there is never -0 (it starts
// as 0.0 plus the first term, and two summands give -0 only when both are
// -0), so adding a zero term leaves it unchanged; what remains is the sum of
// the copied operands in k order, which these helpers form: the same value,
// bit for bit, as the plain sum, for finite operands.
// Row r of F (the constant-velocity transition) applied to the 4-vector v
// with element stride st.
__device__ __forceinline__ double f_row(const double* v, int st, int r)
{
    if (r < 2) return (0.0 + v[r * st]) + v[(r + 2) * st];
    return 0.0 + v[r * st];
}

// Orders one wavefront's LDS operations before and after it (a wait for
// its own outstanding ones); no barrier with the workgroup's other wavefronts.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

struct KModel {  // Q and R of the model (F and H enter through f_row and the written-out products)
    double Q[16];
    double r;
    __device__ KModel(double q, double rr) : r(rr)
    {
        const double qq[16] = {0.25 * q, 0, 0.5 * q, 0, 0, 0.25 * q, 0, 0.5 * q,
                               0.5 * q,  0, q,       0, 0, 0.5 * q,  0, q};
        for (int i = 0; i < 16; ++i) Q[i] = qq[i];
    }
};

__global__ void k_trk_zero(uint32_t* counts, int n, TrkState* st, uint32_t* track_count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counts[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_tracks = 0u;
        st->next_id = 0u;
        st->cur = 0u;
        track_count[0] = 0u;
        track_count[1] = 0u;
    }
}

// per-frame point counts (points outside 0..T-1 are ignored)
__global__ void k_trk_hist(const fz_point* pts, const uint32_t* count, uint32_t cap, int T, uint32_t* counts)
{
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t t = pts[i].t;
        if (t < (uint32_t)T) atomicAdd(&counts[t], 1u);
    }
}

// exclusive scan of counts[0..T) into offs[0..T] and cursor[0..T), one workgroup
__global__ void k_trk_scan(const uint32_t* counts, int T, uint32_t* offs, uint32_t* cursor)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t base;
    if (threadIdx.x == 0) base = 0u;
    __syncthreads();
    for (int c0 = 0; c0 < T; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < T ? counts[i] : 0u;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scan
            const uint32_t a = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
            __syncthreads();
            part[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < T) {
            offs[i] = base + part[threadIdx.x] - v;
            cursor[i] = offs[i];
        }
        __syncthreads();
        if (threadIdx.x == 255) base += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) offs[T] = base;
}

__global__ void k_trk_scatter(const fz_point* pts, const uint32_t* count, uint32_t cap, int T, uint32_t* cursor,
                              int2* bucket)
{
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const fz_point p = pts[i];
        if (p.t >= (uint32_t)T) continue;
        const uint32_t slot = atomicAdd(&cursor[p.t], 1u);
        bucket[slot] = make_int2((int)p.x, (int)p.y);
    }
}

struct Cand {
    double d2;
    int32_t id;
    int16_t ti, pj;
};

// Association order: increasing d2, then track id, then point index.  The
// first part of the key maps d2 (a zero of either sign made +0) to an
// unsigned integer of the same order; the second is (id, point).
__device__ __forceinline__ unsigned long long d2_key(double d2)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(d2 + 0.0);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ unsigned long long idpj_key(const Cand& c)
{
    return (unsigned long long)(uint32_t)c.id << 16 | (uint16_t)c.pj;
}

__device__ __forceinline__ void put_record(fz_track* out, uint32_t k, uint32_t cap, int t, const DevTrack& tr)
{
    if (k < cap) {
        fz_track r;
        r.t = (uint32_t)t;
        r.id = (uint32_t)tr.id;
        r.status = tr.status;
        r.pad = 0;
        r.x = tr.s[0];
        r.y = tr.s[1];
        r.vx = tr.s[2];
        r.vy = tr.s[3];
        out[k] = r;
    }
}

// One workgroup of TRK_WAVES wavefronts marches the frames.  In every
// wavefront each lane owns the tracks lane, lane + 64, ... of the current
// list: it predicts them, tests them against the wavefront's share of the
// frame's points, and later updates them; the wavefronts make the same
// predictions and updates, so each can keep the list's first 64 tracks in its
// registers from frame to frame (passed through LDS when the list is
// compacted); tracks past them live in the workspace.  The first wavefront
// forms the association and writes the list and records; the second sorts the
// next frame's points meanwhile (a frame of up to 64; larger ones are sorted
// by all four at the frame's start).  The
// greedy association is formed in rounds: every candidate that is the first
// (in the (d2, id, point) order) of the remaining candidates of both its track
// and its point is taken, and candidates of taken tracks and points leave;
// for a strict total order this is the matching the one-by-one greedy pass
// makes, in a few rounds instead of one step per candidate.  The next frame's
// points are loaded while the current frame is processed; the record count
// is kept in a register (the first wavefront writes every record).
__global__ __launch_bounds__(TRK_THREADS * TRK_WAVES) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trk_run(const int2* bucket, const uint32_t* offs, int T,
                                                          fz_track_opts o, DevTrack* buf0, DevTrack* buf1,
                                                          uint32_t max_tracks, fz_track* out, uint32_t* count,
                                                          uint32_t cap)
{
    // the frame's points sorted by (y, x), as doubles, for frames of even and
    // odd t (the next frame's are sorted while this one is associated); the
    // candidate search reads them TRK_GROUP at a time, so up to TRK_GROUP - 1
    // past the frame's are read and not used
    __shared__ double2 pts2[2][TRK_MAX_POINTS + TRK_GROUP];
    __shared__ long long skey[TRK_THREADS];  // sort keys of a frame of at most 64 points
    // the gated candidates of the frame; the same memory holds a frame's
    // points as loaded before they are sorted, and after the association the
    // next list's first 64 tracks
    __shared__ union {
        Cand cand[TRK_MAX_CANDS + TRK_THREADS];  // the last 64: one discard slot per lane
        int2 pin[TRK_MAX_POINTS];                // a frame of more than 64 points as loaded
        DevTrack stage[TRK_THREADS];
    } cu;
    __shared__ uint8_t ptaken[TRK_MAX_POINTS];
    __shared__ uint8_t calive[TRK_MAX_CANDS];          // candidate still open (association rounds)
    __shared__ int16_t tmatch[FZ_TRACK_MAX_TRACKS];    // point matched to each track, -1 none
    // first open candidate of each track and point in a round: d2 key, then (id, point) key
    __shared__ unsigned long long tb_d[FZ_TRACK_MAX_TRACKS], tb_k[FZ_TRACK_MAX_TRACKS];
    __shared__ unsigned long long pb_d[TRK_MAX_POINTS], pb_k[TRK_MAX_POINTS];
    Cand* const cand = cu.cand;
    DevTrack* const stage = cu.stage;
    int2* const pin = cu.pin;
    __shared__ uint32_t s_flags, s_nc;
    const int lane = threadIdx.x & (TRK_THREADS - 1);
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TRK_THREADS);
    const bool w0 = wave == 0;  // the wavefront that associates and writes (and sorts a frame not sorted ahead)
    const KModel M(o.q, o.r);
    DevTrack* cur = buf0;
    DevTrack* nxt = buf1;
    uint32_t ntr = 0, next_id = 0, nrec = 0;
    DevTrack rt;  // track `lane` of the current list (lane < ntr)
    if (threadIdx.x == 0) s_flags = 0u;
    if (max_tracks > (uint32_t)FZ_TRACK_MAX_TRACKS) max_tracks = FZ_TRACK_MAX_TRACKS;
    const uint32_t total = offs[T];
    uint32_t f_lo = offs[0], f_hi = T > 0 ? offs[1] : f_lo;
    int pre_x = 0, pre_y = 0;  // point f_lo + lane (loaded a frame ahead)
    if (f_lo + lane < total) {
        const int2 q = bucket[f_lo + lane];
        pre_x = q.x;
        pre_y = q.y;
    }
    // offs[t + 2] for the 64 frames t of the current window (lane t % 64),
    // loaded when the window starts: a frame reads its successor's bounds
    // from a register.  (Loading the next window ahead kept a load in flight
    // across frames, and moving its register from frame to frame made every
    // frame wait for all its outstanding memory operations, the record
    // stores included; now that wait comes once in 64 frames.)
    uint32_t ow_cur = 0;

    for (int t = 0; t < T; ++t) {
        // the frame's point count, in a scalar register (the compiler cannot
        // tell it is the same in every lane; loops over it then run as scalar loops)
        const uint32_t np_all = (uint32_t)__builtin_amdgcn_readfirstlane((int)(f_hi - f_lo));
        if (np_all > (uint32_t)TRK_MAX_POINTS && threadIdx.x == 0) s_flags |= FZ_TRACK_TOO_MANY_POINTS;
        const uint32_t np = min(np_all, (uint32_t)TRK_MAX_POINTS);
        // 1. the frame's points, sorted by (y, x) (keys are distinct); a frame of
        // at most 64 points after the first was sorted during the previous one
        double2* const pts = pts2[t & 1];
        const bool pre_sorted = t > 0 && np <= (uint32_t)TRK_THREADS;
        const int ax = pre_x, ay = pre_y;  // point f_lo + lane
        if (w0)
            for (uint32_t j = lane; j < np; j += TRK_THREADS) {
                if (np > (uint32_t)TRK_THREADS) pin[j] = j < (uint32_t)TRK_THREADS ? make_int2(ax, ay) : bucket[f_lo + j];
                ptaken[j] = 0;
            }
        // the next frame's bounds and first points, in flight during this frame
        const uint32_t tw = (uint32_t)t & 63u;
        if (tw == 0u) {
            ow_cur = offs[min(t + 2 + lane, T)];
            asm volatile("; window bounds in %0" ::"v"(ow_cur));  // the wait for the load stays in this branch
        }
        const uint32_t n_lo = f_hi, n_hi = t + 2 <= T ? (uint32_t)__builtin_amdgcn_readlane((int)ow_cur, (int)tw) : f_hi;
        if (n_lo + lane < total) {
            const int2 q = bucket[n_lo + lane];
            pre_x = q.x;
            pre_y = q.y;
        }
        if (!pre_sorted) {
            if (np <= (uint32_t)TRK_THREADS) {
                // lane j holds point j: its rank counts the smaller (y, x) keys (y in
                // the high word, x offset by 2^31 in the low word, compared as signed
                // 64-bit integers), read back from LDS sixteen at a time
                const uint32_t klo = (uint32_t)ax ^ 0x80000000u, khi = (uint32_t)ay;
                const long long ka = (long long)(((unsigned long long)khi << 32) | klo);
                if (w0) skey[lane] = (uint32_t)lane < np ? ka : 0x7fffffffffffffffll;  // past np: never smaller
                __syncthreads();
                if (w0) {
                    uint32_t rank = 0;
                    for (uint32_t k0 = 0; k0 < np; k0 += 16) {
                        long long kb[16];
#pragma unroll
                        for (uint32_t q = 0; q < 16; ++q) kb[q] = skey[k0 + q];
#pragma unroll
                        for (uint32_t q = 0; q < 16; ++q) rank += kb[q] < ka ? 1u : 0u;
                    }
                    if ((uint32_t)lane < np) pts[rank] = make_double2((double)ax, (double)ay);
                }
            } else {
                __syncthreads();
                for (uint32_t j = threadIdx.x; j < np; j += TRK_THREADS * TRK_WAVES) {
                    const int2 a = pin[j];
                    uint32_t rank = 0;
#pragma unroll 8
                    for (uint32_t k = 0; k < np; ++k) {
                        const int2 b = pin[k];
                        rank += (b.y < a.y || (b.y == a.y && b.x < a.x)) ? 1u : 0u;
                    }
                    pts[rank] = make_double2((double)a.x, (double)a.y);
                }
            }
        }
        if (threadIdx.x == 0) s_nc = 0u;
        __syncthreads();
        // 2. predict every live track and list its gated candidate pairs.  Every
        // wavefront predicts every track (each keeps the list's first 64 in its
        // registers, and all make the same updates), and takes every fourth group
        // of TRK_GROUP points; a group's pairs get consecutive slots from one LDS
        // count, a pair its rank in the group's ballots
        for (uint32_t c0 = 0; c0 < ntr; c0 += TRK_THREADS) {
            const uint32_t i = c0 + lane;
            const bool act = i < ntr;
            double hs[2] = {0.0, 0.0}, Si[4] = {0.0, 0.0, 0.0, 0.0};
            int32_t id = 0;
            DevTrack tr;
            if (act) {
                if (c0 == 0)
                    tr = rt;
                else
                    tr = cur[i];
                double s1[4], FP[16], Pp[16], HP[8], S[4];
                // s1 = F s, FP = F P, Pp = FP F^T + Q, HP = H Pp, S = HP H^T (+ R below)
                for (int r = 0; r < 4; ++r) s1[r] = f_row(tr.s, 1, r);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) FP[4 * i + j] = f_row(tr.P + j, 4, i);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) Pp[4 * i + j] = f_row(FP + 4 * i, 1, j);
                for (int e = 0; e < 16; ++e) Pp[e] = Pp[e] + M.Q[e];
                for (int e = 0; e < 8; ++e) HP[e] = 0.0 + Pp[e];
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) S[2 * i + j] = 0.0 + HP[4 * i + j];
                S[0] = S[0] + M.r;
                S[3] = S[3] + M.r;
                const double det = S[0] * S[3] - S[1] * S[2];
                Si[0] = S[3] / det;
                Si[1] = -S[1] / det;
                Si[2] = -S[2] / det;
                Si[3] = S[0] / det;
                for (int e = 0; e < 4; ++e) tr.s[e] = s1[e];
                for (int e = 0; e < 16; ++e) tr.P[e] = Pp[e];
                for (int e = 0; e < 4; ++e) tr.Si[e] = Si[e];
                if (c0 == 0) rt = tr;
                tmatch[i] = -1;
                for (int e = 0; e < 2; ++e) hs[e] = 0.0 + s1[e];  // H s1
                id = tr.id;
            }
            // a track past the first 64 is read from the workspace by every
            // wavefront, and its prediction written back by one, once all have read it
            if (c0 > 0) {
                __syncthreads();
                if (act && w0) cur[i] = tr;
            }
            // TRK_GROUP points at a time: their d2 are independent chains of double
            // operations, written out step by step across the group so that each
            // step's operations are in flight together; every lane then stores its
            // pair, those that are not candidates into a slot of their own past the
            // list (as does an overflow), so the group is one straight block
            for (uint32_t j0 = (uint32_t)TRK_GROUP * (uint32_t)wave; j0 < np; j0 += (uint32_t)TRK_GROUP * TRK_WAVES) {
                double2 pv[TRK_GROUP];
                double nu0[TRK_GROUP], nu1[TRK_GROUP], tm[4][TRK_GROUP], d2v[TRK_GROUP];
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) pv[q] = pts[j0 + (uint32_t)q];
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    nu0[q] = pv[q].x - hs[0];
                    nu1[q] = pv[q].y - hs[1];
                }
                // d2 = nu^T S^-1 nu: the terms (nu_a Si_ab) nu_b summed from 0.0 in
                // (a, b) order
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    tm[0][q] = nu0[q] * Si[0];
                    tm[1][q] = nu0[q] * Si[1];
                    tm[2][q] = nu1[q] * Si[2];
                    tm[3][q] = nu1[q] * Si[3];
                }
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    tm[0][q] = tm[0][q] * nu0[q];
                    tm[1][q] = tm[1][q] * nu1[q];
                    tm[2][q] = tm[2][q] * nu0[q];
                    tm[3][q] = tm[3][q] * nu1[q];
                }
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) d2v[q] = 0.0 + tm[0][q];
#pragma unroll
                for (int e = 1; e < 4; ++e)
#pragma unroll
                    for (int q = 0; q < TRK_GROUP; ++q) d2v[q] = d2v[q] + tm[e][q];
                // the gate of the whole group first (one mask each), then the slots:
                // the masks' counts in order give each point's base, a lane's rank
                // in its mask its place
                uint64_t m[TRK_GROUP];
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    const bool in = act && j0 + (uint32_t)q < np;
                    const double dq = in ? d2v[q] : __builtin_huge_val();  // outside: never gated in
                    m[q] = __ballot(dq <= o.gate);
                }
                uint32_t base[TRK_GROUP], ncand = 0;
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    base[q] = ncand;
                    ncand += (uint32_t)__popcll(m[q]);
                }
                uint32_t gbase = 0;
                if (ncand) {
                    if (lane == 0) {
                        gbase = atomicAdd(&s_nc, ncand);
                        if (gbase + ncand > (uint32_t)TRK_MAX_CANDS) atomicOr(&s_flags, (uint32_t)FZ_TRACK_TOO_MANY_CANDIDATES);
                    }
                    gbase = (uint32_t)__builtin_amdgcn_readfirstlane((int)gbase);
                }
#pragma unroll
                for (int q = 0; q < TRK_GROUP; ++q) {
                    const bool pass = (m[q] >> lane) & 1ull;
                    const uint32_t k = gbase + base[q] + __builtin_amdgcn_mbcnt_hi((uint32_t)(m[q] >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m[q], 0u));
                    Cand c;
                    c.d2 = d2v[q];
                    c.id = id;
                    c.ti = (int16_t)i;
                    c.pj = (int16_t)(j0 + (uint32_t)q);
                    cand[min(pass ? k : ~0u, (uint32_t)TRK_MAX_CANDS + (uint32_t)lane)] = c;
                }
            }
        }
        __syncthreads();
        const uint32_t nc = min(s_nc, (uint32_t)TRK_MAX_CANDS);
        // 3. greedy association in rounds: an open candidate that comes first
        // (in the (d2, id, point) order) among the open candidates of both its
        // track and its point is taken; then every candidate of a taken track
        // or point closes.  Up to 64 * TRK_ASSOC_REG candidates, each lane keeps
        // its own (lane, lane + 64, ...) in registers, and the first-of slots of
        // a track or point are cleared when its candidates stay open for another
        // round; beyond that the candidates are read from LDS in every pass.
        // One wavefront forms the association (its passes are ordered by waits on
        // its own LDS operations, no barrier); the others wait at the next barrier.
        const uint32_t np_next = min(n_hi - n_lo, (uint32_t)TRK_MAX_POINTS);  // the next frame's, as it will count them
        if (wave == 1 && t + 1 < T && np_next <= (uint32_t)TRK_THREADS) {
            // the second wavefront sorts the next frame's points (its lanes hold
            // them, loaded at this frame's start) into the other buffer, as the
            // first one does for a frame it sorts itself
            const uint32_t klo = (uint32_t)pre_x ^ 0x80000000u, khi = (uint32_t)pre_y;
            const long long ka = (long long)(((unsigned long long)khi << 32) | klo);
            skey[lane] = (uint32_t)lane < np_next ? ka : 0x7fffffffffffffffll;
            wave_sync();
            uint32_t rank = 0;
            for (uint32_t k0 = 0; k0 < np_next; k0 += 16) {
                long long kb[16];
#pragma unroll
                for (uint32_t q = 0; q < 16; ++q) kb[q] = skey[k0 + q];
#pragma unroll
                for (uint32_t q = 0; q < 16; ++q) rank += kb[q] < ka ? 1u : 0u;
            }
            if ((uint32_t)lane < np_next) pts2[(t + 1) & 1][rank] = make_double2((double)pre_x, (double)pre_y);
        }
        if (w0) {
            if (nc <= (uint32_t)(TRK_ASSOC_REG * TRK_THREADS)) {
                unsigned long long rd[TRK_ASSOC_REG], rk[TRK_ASSOC_REG];
                int rti[TRK_ASSOC_REG], rpj[TRK_ASSOC_REG];
                bool al[TRK_ASSOC_REG];
#pragma unroll
                for (int q = 0; q < TRK_ASSOC_REG; ++q) {
                    const uint32_t c = (uint32_t)lane + (uint32_t)q * TRK_THREADS;
                    al[q] = c < nc;
                    rd[q] = rk[q] = 0ull;
                    rti[q] = rpj[q] = 0;
                    if (al[q]) {
                        const Cand a = cand[c];
                        rd[q] = d2_key(a.d2);
                        rk[q] = idpj_key(a);
                        rti[q] = a.ti;
                        rpj[q] = a.pj;
                        tb_d[a.ti] = tb_k[a.ti] = ~0ull;
                        pb_d[a.pj] = pb_k[a.pj] = ~0ull;
                    }
                }
                // every pass loads what it compares before comparing (loads of a
                // closed pair read its stale slots and are not used), so a pass
                // waits on LDS once
                for (;;) {
                    wave_sync();
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q)
                        if (al[q]) {
                            atomicMin(&tb_d[rti[q]], rd[q]);
                            atomicMin(&pb_d[rpj[q]], rd[q]);
                        }
                    wave_sync();
                    unsigned long long td[TRK_ASSOC_REG], pd[TRK_ASSOC_REG], tk[TRK_ASSOC_REG], pk[TRK_ASSOC_REG];
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q) {
                        td[q] = tb_d[rti[q]];
                        pd[q] = pb_d[rpj[q]];
                    }
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q)
                        if (al[q]) {
                            if (rd[q] == td[q]) atomicMin(&tb_k[rti[q]], rk[q]);
                            if (rd[q] == pd[q]) atomicMin(&pb_k[rpj[q]], rk[q]);
                        }
                    wave_sync();
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q) {
                        tk[q] = tb_k[rti[q]];
                        pk[q] = pb_k[rpj[q]];
                    }
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q) {
                        const bool take = al[q] & (rd[q] == td[q]) & (rk[q] == tk[q]) & (rd[q] == pd[q]) & (rk[q] == pk[q]);
                        if (take) {
                            tmatch[rti[q]] = (int16_t)rpj[q];
                            ptaken[rpj[q]] = 1;
                        }
                    }
                    wave_sync();
                    int tmq[TRK_ASSOC_REG], ptq[TRK_ASSOC_REG];
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q) {
                        tmq[q] = tmatch[rti[q]];
                        ptq[q] = ptaken[rpj[q]];
                    }
                    bool open = false;
#pragma unroll
                    for (int q = 0; q < TRK_ASSOC_REG; ++q)
                        if (al[q]) {
                            if (tmq[q] >= 0 || ptq[q]) {
                                al[q] = false;
                            } else {
                                open = true;
                                tb_d[rti[q]] = tb_k[rti[q]] = ~0ull;
                                pb_d[rpj[q]] = pb_k[rpj[q]] = ~0ull;
                            }
                        }
                    if (!__any(open)) break;
                }
            } else {
                // the same passes over the LDS list (slots cleared before the first
                // round and, for candidates still open, in the pass that closes the others)
                for (uint32_t c = lane; c < nc; c += TRK_THREADS) {
                    calive[c] = 1;
                    const Cand a = cand[c];
                    tb_d[a.ti] = tb_k[a.ti] = ~0ull;
                    pb_d[a.pj] = pb_k[a.pj] = ~0ull;
                }
                for (;;) {
                    wave_sync();
                    for (uint32_t c = lane; c < nc; c += TRK_THREADS)
                        if (calive[c]) {
                            const Cand a = cand[c];
                            const unsigned long long d = d2_key(a.d2);
                            atomicMin(&tb_d[a.ti], d);
                            atomicMin(&pb_d[a.pj], d);
                        }
                    wave_sync();
                    for (uint32_t c = lane; c < nc; c += TRK_THREADS)
                        if (calive[c]) {
                            const Cand a = cand[c];
                            const unsigned long long d = d2_key(a.d2), k = idpj_key(a);
                            const unsigned long long td = tb_d[a.ti], pd = pb_d[a.pj];
                            if (d == td) atomicMin(&tb_k[a.ti], k);
                            if (d == pd) atomicMin(&pb_k[a.pj], k);
                        }
                    wave_sync();
                    for (uint32_t c = lane; c < nc; c += TRK_THREADS)
                        if (calive[c]) {
                            const Cand a = cand[c];
                            const unsigned long long d = d2_key(a.d2), k = idpj_key(a);
                            const unsigned long long td = tb_d[a.ti], tk = tb_k[a.ti], pd = pb_d[a.pj], pk = pb_k[a.pj];
                            if ((d == td) & (k == tk) & (d == pd) & (k == pk)) {
                                tmatch[a.ti] = a.pj;
                                ptaken[a.pj] = 1;
                            }
                        }
                    wave_sync();
                    bool open = false;
                    for (uint32_t c = lane; c < nc; c += TRK_THREADS)
                        if (calive[c]) {
                            const Cand a = cand[c];
                            const int tm = tmatch[a.ti], pt = ptaken[a.pj];
                            if (tm >= 0 || pt) {
                                calive[c] = 0;
                            } else {
                                open = true;
                                tb_d[a.ti] = tb_k[a.ti] = ~0ull;
                                pb_d[a.pj] = pb_k[a.pj] = ~0ull;
                            }
                        }
                    if (!__any(open)) break;
                }
            }
        }
        __syncthreads();
        // 5. update or count a miss; survivors to the next list in id order, with their records
        uint32_t n_alive = 0;
        for (uint32_t c0 = 0; c0 < ntr; c0 += TRK_THREADS) {
            const uint32_t i = c0 + lane;
            DevTrack tr;
            bool alive = false;
            if (i < ntr) {
                if (c0 == 0)
                    tr = rt;
                else
                    tr = cur[i];
                const int j = tmatch[i];
                if (j >= 0) {
                    double hs[2], nu[2], PHt[8], K[8], Knu[4], KH[16], IKH[16], Pn[16];
                    for (int e = 0; e < 2; ++e) hs[e] = 0.0 + tr.s[e];  // H s
                    nu[0] = pts[j].x - hs[0];
                    nu[1] = pts[j].y - hs[1];
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 2; ++b) PHt[2 * a + b] = 0.0 + tr.P[4 * a + b];  // P H^T
                    mm<4, 2, 2>(PHt, tr.Si, K);
                    mm<4, 2, 1>(K, nu, Knu);
                    for (int e = 0; e < 4; ++e) tr.s[e] = tr.s[e] + Knu[e];
                    for (int a = 0; a < 4; ++a)  // K H: columns 0, 1 of K, then zeros
                        for (int b = 0; b < 4; ++b) KH[4 * a + b] = b < 2 ? 0.0 + K[2 * a + b] : 0.0;
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b) IKH[4 * a + b] = (a == b ? 1.0 : 0.0) - KH[4 * a + b];
                    // (I - KH) P: columns 2 and 3 of I - KH are those of the identity
                    // (1 - 0 and 0 - 0 exactly), so rows 2 and 3 add P's own row
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b) {
                            const double acc = (0.0 + IKH[4 * a] * tr.P[b]) + IKH[4 * a + 1] * tr.P[4 + b];
                            Pn[4 * a + b] = a < 2 ? acc : acc + tr.P[4 * a + b];
                        }
                    for (int e = 0; e < 16; ++e) tr.P[e] = Pn[e];
                    tr.miss = 0;
                    tr.status = 1;
                } else {
                    tr.miss += 1;
                    tr.status = 0;
                }
                alive = tr.miss <= o.max_miss;
            }
            const uint64_t m = __ballot(alive);
            const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (alive && w0) {
                const uint32_t pos = n_alive + before;
                if (pos < (uint32_t)TRK_THREADS)
                    stage[pos] = tr;
                else
                    nxt[pos] = tr;
                put_record(out, nrec + before, cap, t, tr);
            }
            n_alive += (uint32_t)__popcll(m);
            nrec += (uint32_t)__popcll(m);
        }
        // 6. every point left over starts a track (ids in point order)
        uint32_t n_new = 0;
        for (uint32_t c0 = 0; c0 < np; c0 += TRK_THREADS) {
            const uint32_t j = c0 + lane;
            const bool fresh = j < np && !ptaken[j];
            const uint32_t before = (uint32_t)__popcll(__ballot(fresh) & ((1ull << lane) - 1ull));
            const uint32_t pos = n_alive + n_new + before;
            const bool keep = fresh && pos < max_tracks;
            if (fresh && !keep && w0) atomicOr(&s_flags, (uint32_t)FZ_TRACK_TOO_MANY_TRACKS);
            const uint64_t m = __ballot(keep);
            if (keep && w0) {
                DevTrack tr;
                tr.id = (int32_t)(next_id + n_new + before);
                tr.miss = 0;
                tr.status = 2;
                tr.pad = 0;
                tr.s[0] = pts[j].x;
                tr.s[1] = pts[j].y;
                tr.s[2] = 0.0;
                tr.s[3] = 0.0;
                for (int e = 0; e < 16; ++e) tr.P[e] = 0.0;
                tr.P[0] = o.r;
                tr.P[5] = o.r;
                tr.P[10] = o.v0;
                tr.P[15] = o.v0;
                for (int e = 0; e < 4; ++e) tr.Si[e] = 0.0;
                if (pos < (uint32_t)TRK_THREADS)
                    stage[pos] = tr;
                else
                    nxt[pos] = tr;
                put_record(out, nrec + (uint32_t)__popcll(m & ((1ull << lane) - 1ull)), cap, t, tr);
            }
            nrec += (uint32_t)__popcll(m);
            n_new += (uint32_t)__popcll(__ballot(fresh));
        }
        next_id += n_new;
        ntr = min(n_alive + n_new, max_tracks);
        DevTrack* sw = cur;
        cur = nxt;
        nxt = sw;
        __syncthreads();
        if ((uint32_t)lane < ntr) rt = stage[lane];
        f_lo = n_lo;
        f_hi = n_hi;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        count[0] = nrec;
        atomicOr(&count[1], s_flags);
    }
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t track_workspace_bytes(int T, uint32_t point_capacity, uint32_t max_tracks)
{
    return align256(sizeof(TrkState)) + 3 * align256(sizeof(uint32_t) * ((size_t)T + 1)) +
           align256(sizeof(int2) * (size_t)point_capacity) + 2 * align256(sizeof(DevTrack) * (size_t)max_tracks);
}

fz_status track_points(const fz_point* d_points, const uint32_t* d_count, uint32_t cap, int T, const fz_track_opts& o,
                       fz_track* d_tracks, uint32_t* d_track_count, uint32_t track_cap, void* ws, void* stream)
{
    (void)hipGetLastError();
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    TrkState* st = (TrkState*)w;
    w += align256(sizeof(TrkState));
    uint32_t* counts = (uint32_t*)w;
    w += align256(sizeof(uint32_t) * ((size_t)T + 1));
    uint32_t* offs = (uint32_t*)w;
    w += align256(sizeof(uint32_t) * ((size_t)T + 1));
    uint32_t* cursor = (uint32_t*)w;
    w += align256(sizeof(uint32_t) * ((size_t)T + 1));
    int2* bucket = (int2*)w;
    w += align256(sizeof(int2) * (size_t)cap);
    DevTrack* b0 = (DevTrack*)w;
    w += align256(sizeof(DevTrack) * (size_t)o.max_tracks);
    DevTrack* b1 = (DevTrack*)w;
    const unsigned gz = (unsigned)std::min<size_t>(((size_t)T + 256) / 256, 1024);
    hipLaunchKernelGGL(k_trk_zero, dim3(gz), dim3(256), 0, s, counts, T + 1, st, d_track_count);
    const unsigned gp = (unsigned)std::max<size_t>(1, std::min<size_t>(((size_t)cap + 255) / 256, 1024));
    if (cap > 0) hipLaunchKernelGGL(k_trk_hist, dim3(gp), dim3(256), 0, s, d_points, d_count, cap, T, counts);
    hipLaunchKernelGGL(k_trk_scan, dim3(1), dim3(256), 0, s, counts, T, offs, cursor);
    if (cap > 0)
        hipLaunchKernelGGL(k_trk_scatter, dim3(gp), dim3(256), 0, s, d_points, d_count, cap, T, cursor, bucket);
    hipLaunchKernelGGL(k_trk_run, dim3(1), dim3(TRK_THREADS * TRK_WAVES), 0, s, bucket, offs, T, o, b0, b1,
                       (uint32_t)o.max_tracks, d_tracks, d_track_count, track_cap);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("fz_track_points: launch: ") + hipGetErrorString(e));
    return FZ_OK;
}

}  // namespace fz

using namespace fz;

extern "C" {

fz_status fz_track_default_opts(fz_track_opts* out)
{
    if (!out) return fail(FZ_E_INVALID, "fz_track_default_opts: null output");
    out->q = 0.5;
    out->r = 1.0;
    out->gate = 9.21;
    out->v0 = 4.0;
    out->max_miss = 3;
    out->max_tracks = FZ_TRACK_MAX_TRACKS;
    return FZ_OK;
}

static fz_status check_opts(const fz_track_opts* o, const char* who)
{
    if (!o) return fail(FZ_E_INVALID, std::string(who) + ": null options");
    if (!(o->q >= 0.0 && o->r > 0.0 && o->gate >= 0.0 && o->v0 >= 0.0) || !std::isfinite(o->q) ||
        !std::isfinite(o->r) || !std::isfinite(o->gate) || !std::isfinite(o->v0))
        return fail(FZ_E_INVALID, std::string(who) + ": need q >= 0, r > 0, gate >= 0, v0 >= 0, all finite");
    if (o->max_miss < 0 || o->max_tracks < 1 || o->max_tracks > FZ_TRACK_MAX_TRACKS)
        return fail(FZ_E_INVALID, std::string(who) + ": need max_miss >= 0 and max_tracks in [1, 4096]");
    return FZ_OK;
}

size_t fz_track_workspace_bytes(int32_t frames, uint32_t point_capacity, const fz_track_opts* opts)
{
    if (frames <= 0 || check_opts(opts, "fz_track_workspace_bytes") != FZ_OK) return 0;
    return track_workspace_bytes(frames, point_capacity, (uint32_t)opts->max_tracks);
}

fz_status fz_track_points(const fz_point* d_points, const uint32_t* d_point_count, uint32_t point_capacity,
                          int32_t frames, const fz_track_opts* opts, fz_track* d_tracks, uint32_t* d_track_count,
                          uint32_t track_capacity, void* d_workspace, size_t ws_bytes, void* stream)
{
    const fz_status st = check_opts(opts, "fz_track_points");
    if (st != FZ_OK) return st;
    if (frames <= 0) return fail(FZ_E_INVALID, "fz_track_points: frames must be positive");
    if (!d_point_count || !d_track_count || (point_capacity > 0 && !d_points) || (track_capacity > 0 && !d_tracks))
        return fail(FZ_E_INVALID, "fz_track_points: null buffer");
    const size_t need = track_workspace_bytes(frames, point_capacity, (uint32_t)opts->max_tracks);
    if (!d_workspace || ws_bytes < need)
        return fail(FZ_E_WORKSPACE, "fz_track_points: workspace needs " + std::to_string(need) + " bytes");
    return track_points(d_points, d_point_count, point_capacity, frames, *opts, d_tracks, d_track_count,
                        track_capacity, d_workspace, stream);
}

}  // extern "C"
