/*
 * fz -- fused video-kernel chains on MI355X (gfx950).
 *
 * C ABI of the library.  It implements the method of "Efficient Kernel Fusion
 * Techniques for Massive Video Data Analysis on GPGPUs" (Adnan, Radhakrishnan,
 * Karabuk): a sequence of image kernels K_1..K_n applied in order to a video
 * volume N x M x T (Sec. III) is split into contiguous groups, each group run as
 * one fused kernel that loads its input box once, keeps every intermediate
 * on chip and stores only its last output (Sec. V-B, Eq. 2; Sec. VI-B,
 * Algorithm 1).  The split is the one with the least predicted cost under the
 * on-chip memory budget (Sec. VI-A, Fig. 5).
 *
 * Conventions for every call:
 *   - All device pointers are caller-owned device memory (hipMalloc'd or a
 *     PyTorch CUDA tensor's data_ptr()); the library never frees them and
 *     allocates no device memory on the run path.
 *   - Host pointers are read during the call only, unless stated.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Runs are asynchronous on that stream; all argument checks happen on the
 *     host before the first launch, so an error return means nothing was
 *     launched.
 *   - Errors are reported by the return code; fz_last_error() gives a
 *     human-readable message for the calling thread's last failed call.
 *
 * Video layouts (frame-major, row-major, x along the width):
 *   u8 gray / mask:      [T][H][W]
 *   u8 RGB:              [T][H][W][3] interleaved
 *   f32, c channels:     [c][T][H][W] planar
 */
#ifndef FZ_H
#define FZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fz_status;
enum {
    FZ_OK = 0,
    FZ_E_INVALID = 1,     /* null pointer, bad size, malformed or unsupported chain */
    FZ_E_LDS = 2,         /* some stage cannot fit the on-chip (LDS) budget even alone */
    FZ_E_HIP = 3,         /* a HIP launch or query failed; see fz_last_error() */
    FZ_E_WORKSPACE = 4,   /* workspace smaller than fz_workspace_bytes() */
    FZ_E_UNSUPPORTED = 5  /* valid request this build does not implement */
};

/* Image operations.  Table II of the paper classifies the operations of its
 * tracking pipeline as point, rectangular and multi-frame operations (Table I
 * gives the classes by the extent of the input window); the Harris-corner
 * chain below is built from the same classes. */
enum {
    FZ_OP_RGB2GRAY = 1,   /* point op: u8 RGB -> u8 gray, floor((299R+587G+114B+500)/1000) */
    FZ_OP_GAUSS5 = 2,     /* rectangular, radius 2: u8 -> f32, sampled Gaussian, param[0] = sigma */
    FZ_OP_SOBEL3 = 3,     /* rectangular, radius 1: f32 -> 2 x f32 (Ix, Iy), unnormalised */
    FZ_OP_GRADMAG = 4,    /* point op: 2 x f32 -> f32, sqrt(Ix^2 + Iy^2) */
    FZ_OP_PRODUCTS = 5,   /* point op: 2 x f32 -> 3 x f32 (Ix^2, Ix*Iy, Iy^2) */
    FZ_OP_BOXSUM5 = 6,    /* rectangular, radius 2: 3 x f32 -> 3 x f32, 5x5 window sums */
    FZ_OP_HARRIS = 7,     /* point op: 3 x f32 -> f32, Sxx*Syy - Sxy^2 - k (Sxx+Syy)^2, param[0] = k */
    FZ_OP_THRESHOLD = 8,  /* point op: f32 -> f32, v >= param[0] ? v : 0 */
    FZ_OP_NMS3 = 9,       /* rectangular, radius 1: f32 -> u8 mask (255 = feature) + feature points */
    FZ_OP_FRAMEDIFF = 10, /* multi-frame point op, 1 frame back: u8 -> u8, |m[t] - m[t-1]| (m[-1] = m[0]) */

    /* Generic single-channel stages: the Table I classes with free parameters.
     * A chain is either a contiguous part of the Harris chain above
     * (FZ_OP_RGB2GRAY .. FZ_OP_FRAMEDIFF in that order, or FZ_OP_GAUSS5,
     * FZ_OP_SOBEL3, FZ_OP_GRADMAG) or made of generic stages only.  Generic
     * stages read u8 (first stage only) or f32 and write f32, one channel;
     * window reads use replicate borders. */
    FZ_OP_STENCIL = 11,   /* rectangular, radii rx, ry in [0, 3]: out(x,y) = sum_{v,u} w[v+ry][u+rx] in(x+u, y+v),
                             `weights` = (2ry+1) x (2rx+1) floats, row-major; summed in row order v = -ry..ry,
                             each row u = -rx..rx, by fused multiply-adds from 0.
                             Spatio-temporal (Table I) when rt in [1, 3]: the stencil also reads the rt frames
                             before t, out(x,y,t) = sum_{tau=0..rt} sum_{v,u} w[tau][v+ry][u+rx] in(x+u, y+v, t-tau)
                             with frames before the first replicating the first; `weights` then holds
                             (rt+1) x (2ry+1) x (2rx+1) floats (tau = 0 is the current frame), summed frame by
                             frame from tau = 0, each frame as above, one multiply-add chain */
    FZ_OP_BOX = 12,       /* rectangular, radii rx, ry in [0, 3]: unweighted window sum; each row summed
                             left to right, the row sums added top to bottom */
    FZ_OP_POINT = 13,     /* point op: param[0] = FZ_POINT_* kind, param[1] = a, param[2] = b */
    FZ_OP_IIR = 14        /* multi-frame point op (Table II "IIR filter"), rt = -1 (every earlier frame):
                             y[t] = a x[t] + (1 - a) y[t-1] per pixel with y[-1] := x[0], param[0] = a in (0, 1];
                             the state and fma(a, x, (1 - a) y_prev) in double precision, each output rounded
                             once to f32.  A group holding an IIR marches every frame of the clip in order */
};

/* Kinds of FZ_OP_POINT. */
enum {
    FZ_POINT_AFFINE = 0,  /* fmaf(a, v, b) */
    FZ_POINT_ABS = 1,     /* |v| */
    FZ_POINT_SQUARE = 2,  /* v * v */
    FZ_POINT_SQRTABS = 3, /* sqrt(|v|), correctly rounded */
    FZ_POINT_CLAMP = 4    /* min(max(v, a), b), a <= b */
};

enum { FZ_U8 = 1, FZ_F32 = 2 };

/* Dependence of a stage on its predecessor (Sec. V-A): thread-to-thread (the
 * same pixel), thread-to-multi-thread (a window of pixels of the same block),
 * kernel-to-kernel (pixels of other blocks: never fused with its predecessor). */
enum { FZ_DEP_TT = 0, FZ_DEP_TMT = 1, FZ_DEP_KK = 2 };

/* Access pattern and parameters of one stage (Sec. IV: an output pixel reads a
 * (2rx+1) x (2ry+1) window of its input over rt+1 frames).  Fill it with
 * fz_stage_describe() and change param[] as needed; the planner rejects a
 * descriptor whose pattern disagrees with the operation. */
typedef struct fz_stage {
    int32_t op;
    int32_t rx, ry, rt;
    int32_t in_ch, out_ch;
    int32_t in_dtype, out_dtype;
    int32_t dep;
    float param[4];
    const float* weights;  /* FZ_OP_STENCIL: host array, copied by fz_plan_chain; NULL otherwise */
} fz_stage;

/* Feature point emitted by FZ_OP_NMS3 (frame, row, column, corner response). */
typedef struct fz_point {
    uint32_t t, y, x;
    float response;
} fz_point;

enum { FZ_PART_OPTIMAL = 0, FZ_PART_UNFUSED = 1, FZ_PART_EXPLICIT = 2 };
enum { FZ_COST_ANALYTIC = 0, FZ_COST_LEARNED = 1, FZ_COST_MEASURED = 2 };

typedef struct fz_plan_opts {
    int32_t width, height, frames;  /* video size the plan is made for (> 0) */
    int32_t lds_budget_bytes;       /* on-chip budget per fused kernel; 0 = 163840 (160 KB per CU) */
    int32_t partition;              /* FZ_PART_*: optimal (planner), one kernel per stage, or explicit */
    int32_t n_cuts;                 /* FZ_PART_EXPLICIT: number of entries in cuts */
    const int32_t* cuts;            /* FZ_PART_EXPLICIT: last stage index of every group but the final,
                                       strictly increasing, each in [0, n-2] */
    int32_t cost_model;             /* FZ_COST_ANALYTIC (bytes), FZ_COST_LEARNED (predicted microseconds) or
                                       FZ_COST_MEASURED (planned with bytes; fz_plan_measure then
                                       replaces the prices with measured microseconds) */
    int32_t tile_w, tile_h;         /* output box of one workgroup; 0 = planner's choice */
    int32_t frames_per_block;       /* frames one workgroup marches through; 0 = planner's choice */
    int32_t engine;                 /* FZ_ENGINE_*: kernel family for groups that have a choice */
    const float* cost_weights;      /* FZ_COST_LEARNED: host copy of the trained cost network's parameters
                                       (fz_mlp_param_count(fz_cost_n_features()) floats, layout of
                                       fz_mlp_forward); read during fz_plan_chain only */
    int32_t cost_n_features;        /* FZ_COST_LEARNED: must equal fz_cost_n_features() */
} fz_plan_opts;

/* Kernel families.  TILE: a workgroup loads its halo box into LDS and runs the
 * group's stages there (any group).  ROW: a wavefront marches down a strip of
 * columns keeping each stage's live rows in registers (the Harris chain from
 * the Gaussian or the gray conversion to the suppression or the frame
 * difference, frames at least 128 pixels wide).  AUTO picks ROW where it
 * applies, TILE elsewhere.  JIT (generic chains only; Sec. X's generated
 * fused kernels): each generic group with a window stage gets a kernel
 * written out for its stage list -- radii, box sizes, frame rings and weights
 * as constants, point and IIR stages inline -- compiled for gfx950 with hipRTC
 * when the plan is made (a compile error fails fz_plan_chain), loaded on each
 * device at its first run and cached for the process; tiles 16x16, 32x16,
 * 32x32, 64x16, 64x32; a work item marches frames_per_block frames (up to 4
 * by default for a group without temporal stages).  Its output equals TILE's
 * in value (the sign of a zero sum aside).  Point-only groups of a JIT plan
 * run as in AUTO. */
enum { FZ_ENGINE_AUTO = 0, FZ_ENGINE_TILE = 1, FZ_ENGINE_ROW = 2, FZ_ENGINE_STREAM = 3, FZ_ENGINE_JIT = 4 };

typedef struct fz_plan fz_plan;  /* opaque, host memory */

/* Per-group description of a plan. */
typedef struct fz_segment_info {
    int32_t first, last;            /* stage indices covered by this fused kernel */
    int32_t tile_w, tile_h;         /* output box x, y (Sec. V, Fig. 3); ROW: strip span, band rows */
    int32_t frames_per_block;       /* output box t */
    int32_t halo, halo_t;           /* input-box growth per side in x/y, and in frames (Sec. VI-C) */
    int32_t lds_bytes;              /* on-chip memory of one workgroup */
    int32_t streaming;              /* 1 = no window stage: one pass, no on-chip staging */
    int32_t engine;                 /* FZ_ENGINE_TILE, FZ_ENGINE_ROW or FZ_ENGINE_STREAM */
    double bytes_per_px;            /* compulsory global-memory bytes per output pixel */
    double cost;                    /* the planner's cost of this group */
} fz_segment_info;

/* Fill `out` with the access pattern and default parameters of `op`
 * (sigma 1, k 0.04, threshold 1e8; generic stages: f32 in and out, radius 1
 * for FZ_OP_STENCIL and FZ_OP_BOX with no weights set, the identity
 * FZ_POINT_AFFINE a = 1, b = 0 for FZ_OP_POINT).  FZ_E_INVALID for an
 * unknown op. */
fz_status fz_stage_describe(int32_t op, fz_stage* out);

/* Box sizing of Sec. VI-E (Eq. 6): of the boxes x * x * t with x^2 t = beta
 * (pixels), the one whose input box (x + 2 dx)^2 (t + dt) is least, for a halo
 * of dx pixels per side and dt frames: x = cbrt(2 beta dx / dt),
 * t = cbrt(beta) (dt / dx)^(2/3) / 2^(2/3).  With dt = 0 the flattest box
 * (t = 1, x = sqrt(beta)); with dx = 0 the thinnest (x = 1, t = beta).
 * The planner uses it for the frame run of groups with a stencil that looks
 * back, with beta = W H T / 1024 output pixels per work item (the work items
 * that fill the device).  FZ_E_INVALID for beta <= 0 or a negative halo. */
fz_status fz_box_eq6(double beta, double dx, double dt, double* x, double* t);

/* Plan a chain (Sec. VI-A): validate the n stage descriptors (host array),
 * split them into fusable sets at kernel-to-kernel dependences, price every
 * contiguous group, and pick the partition of least total cost (ties: fewer
 * groups, then later cuts).  The analytic cost of a group is its compulsory
 * global-memory traffic (Eq. 2 applied per group; Sec. VI-D); a group whose
 * smallest tile does not fit `lds_budget_bytes` is not allowed.  On success
 * *out owns a new plan the caller frees with fz_plan_destroy().  The chain must
 * be a contiguous part of  rgb2gray, gauss5, sobel3, products, boxsum5,
 * harris, threshold, nms3, framediff  or of  gauss5, sobel3, gradmag, or a
 * sequence of generic stages (FZ_OP_STENCIL / FZ_OP_BOX / FZ_OP_POINT /
 * FZ_OP_IIR; a window stage must declare FZ_DEP_TMT or FZ_DEP_KK); other
 * sequences give FZ_E_UNSUPPORTED.  Stencil weights must be finite and are
 * copied.  A group's stencils may hold at most 784 weights in all (over every
 * frame they read); larger groups are not formed.  Chains with temporal
 * generic stages (an IIR, a stencil with rt > 0) cannot use FZ_COST_LEARNED
 * (FZ_E_UNSUPPORTED: the cost network was not trained on them), and a
 * frames_per_block request below the clip length is refused for a group that
 * holds an IIR. */
fz_status fz_plan_chain(const fz_stage* stages, int32_t n, const fz_plan_opts* opts, fz_plan** out);

void fz_plan_destroy(fz_plan* plan);

int32_t fz_plan_num_segments(const fz_plan* plan);
/* Copy the last stage index of each group into seg_last[0..cap). */
fz_status fz_plan_segments(const fz_plan* plan, int32_t* seg_last, int32_t cap);
fz_status fz_plan_segment_info(const fz_plan* plan, int32_t i, fz_segment_info* out);
/* Override the kernel configuration of group i (autotuning): engine
 * (FZ_ENGINE_TILE / FZ_ENGINE_ROW / FZ_ENGINE_AUTO), tile_w x tile_h for the
 * tile engine (a compiled tile) or tile_h = rows per band for the row engine,
 * frames_per_block (0 = the planner's choice).  The group is re-priced with the
 * analytic model; FZ_E_UNSUPPORTED if the configuration does not exist for the
 * group, FZ_E_LDS if it does not fit the plan's budget.  A cached batch graph
 * is dropped. */
fz_status fz_plan_set_segment_config(fz_plan* plan, int32_t i, int32_t engine, int32_t tile_w, int32_t tile_h,
                                     int32_t frames_per_block);

/* Planner objective of the chosen partition (bytes for the analytic model). */
double fz_plan_cost(const fz_plan* plan);
/* The planner's price of the group a..b (inclusive); +inf if not allowed. */
fz_status fz_plan_group_cost(const fz_plan* plan, int32_t a, int32_t b, double* cost);

/* Solve the partition model of Fig. 5 for an arbitrary price table: cost is an
 * n x n row-major host array, cost[a*n+b] = price of fusing a..b (a <= b;
 * +inf = not allowed; entries below the diagonal are ignored).  Writes the
 * last stage of each group to seg_last (capacity n), their number to *n_seg
 * and the optimum to *total (+inf if nothing is feasible).  Exact: the
 * contiguous-group model is a shortest path over cut positions.  n in [1, 64]. */
fz_status fz_partition_min(const double* cost, int32_t n, int32_t* seg_last, int32_t* n_seg, double* total);

/* Device workspace a run needs: the intermediates between groups, the IIR
 * checkpoints of a group whose leading IIRs resume at frame runs, and the
 * frame-boundary exchange of a frame-difference group on the Harris row
 * kernel (two areas of 8 * K bytes per band row and one counter per boundary
 * between runs of one strip and band; cleared by the run itself). */
size_t fz_workspace_bytes(const fz_plan* plan);

/* Measured prices (Sec. VI-A: the price of a candidate fused kernel is its
 * execution time).  Runs every contiguous group of the plan in every kernel
 * configuration it can run in (the planner's choice and each compiled tile)
 * on the device: the groups starting at stage a read the chain's real input
 * of stage a, made from d_in (the plan's input video, caller-owned, layout of
 * fz_run_chain) by the stages before a.  Each configuration runs once untimed
 * and `reps` (1..1000) times bracketed by HIP events on `stream`; its price
 * is the median in microseconds.  Then each group takes its fastest
 * configuration and the partition becomes the exact optimum over those
 * prices (fz_plan_cost returns microseconds from then on), whatever partition
 * mode the plan was made with.  d_workspace: caller-owned device memory of at
 * least fz_measure_workspace_bytes() bytes (three buffers of the largest
 * stage output and a counter); its contents are scratch.  Blocks until the
 * stream has drained.  FZ_E_WORKSPACE if the workspace is too small (checked
 * before any launch), FZ_E_HIP on a failed launch or event call; the plan is
 * unchanged unless FZ_OK is returned.  A cached batch graph is dropped. */
size_t fz_measure_workspace_bytes(const fz_plan* plan);
fz_status fz_plan_measure(fz_plan* plan, const void* d_in, void* d_workspace, size_t ws_bytes, int32_t reps,
                          void* stream);

/* Run the planned chain on the device (Sec. VI-B, Algorithm 1 per group):
 *   d_in:   input video in the layout of the first stage's input type
 *   d_out:  output video in the layout of the last stage's output type
 *   d_points, d_point_count, point_capacity: feature points of FZ_OP_NMS3
 *           (may be NULL/0 if the chain has no nms3 stage).  *d_point_count is
 *           reset by the run and counts every point, also past the capacity;
 *           read it after the stream has synchronised and compare.  Point order
 *           is unspecified.
 *   d_workspace, ws_bytes: at least fz_workspace_bytes(plan) bytes.
 * The output equals that of the plain sequence whatever the partition. */
fz_status fz_run_chain(const fz_plan* plan, const void* d_in, void* d_out, fz_point* d_points,
                       uint32_t* d_point_count, uint32_t point_capacity, void* d_workspace,
                       size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same run
 * as fz_run_chain, with the workspace for intermediates between groups taken
 * from a fixed device array inside the library instead of a caller buffer.
 * The caller still owns d_in, d_out, d_points and d_point_count (meanings as
 * in fz_run_chain).  The call itself allocates nothing.
 *   - Limit: plans whose fz_workspace_bytes() exceeds FZ_STATIC_WORKSPACE_BYTES
 *     (64 MiB) are refused with FZ_E_WORKSPACE before anything is launched or
 *     any device is touched (the fused 800x600x1000 RGB chain at its planned
 *     2-frame runs needs 67 MB of exchange words: plan it with longer runs,
 *     fz_plan_set_segment_config, to run it here).
 *   - Each GPU the library runs on holds its own 64 MiB array from the first
 *     call on that device (which looks its address up) until the process ends.
 *   - Every call on one GPU shares that GPU's array and leaves its contents
 *     behind: calls that overlap in time on one device (two streams or two
 *     host threads) race on it and must be serialised by the caller.
 * Runs on the current device; FZ_E_HIP if the array's address cannot be
 * found. */
#define FZ_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
fz_status fz_run_chain_static(const fz_plan* plan, const void* d_in, void* d_out, fz_point* d_points,
                              uint32_t* d_point_count, uint32_t point_capacity, void* stream);

/* One clip of a batch: its own input, output, size and feature-point buffer. */
typedef struct fz_clip {
    const void* d_in;               /* input video, layout of the plan's first stage */
    void* d_out;                    /* output video, layout of the plan's last stage */
    int32_t width, height, frames;  /* > 0 */
    fz_point* d_points;             /* may be NULL (then capacity must be 0) */
    uint32_t* d_point_count;        /* may be NULL; reset by the run, counts past the capacity */
    uint32_t point_capacity;
} fz_clip;

/* Device workspace fz_run_batch() needs for these clips. */
size_t fz_batch_workspace_bytes(const fz_plan* plan, const fz_clip* clips, int32_t n_clips);

/* Run the plan's chain and partition over n_clips clips of possibly different
 * sizes and lengths (host array of descriptors).  Every clip's output and point
 * set equal those of fz_run_chain on that clip alone.  When the plan is a single
 * group the row kernel implements, all clips go through one persistent launch
 * whose wavefronts take (clip, strip, band, frame run) work items from a queue;
 * otherwise the clips' groups are launched clip after clip.  The launches are
 * captured once into a HIP graph, kept in the plan and replayed while the clip
 * descriptors and workspace pointer stay the same (they are compared on every
 * call; a change re-captures).  A plan must not run batches on two streams at
 * once.  n_clips in [1, 1024]. */
fz_status fz_run_batch(fz_plan* plan, const fz_clip* clips, int32_t n_clips, void* d_workspace, size_t ws_bytes,
                       void* stream);

/* ---------------------------------------------------------------- tracking
 * The paper's pipeline ends by applying a Kalman filter to the extracted
 * feature points (Sec. III; Table II "Apply Kalman Filter": single point,
 * multi-frame); Table IV marks it kernel-to-kernel dependent, so it is never
 * fused with the kernels before it.  fz_track_points runs it on the point
 * list a chain's FZ_OP_NMS3 stage produced (its own launches, after the
 * chain, on the same stream).  The paper gives no model; this one is the
 * discrete Kalman filter with a constant-velocity state s = (x, y, vx, vy)
 * (column, row, pixels per frame):
 *   F = [[1,0,1,0],[0,1,0,1],[0,0,1,0],[0,0,0,1]],
 *   Q = q [[1/4,0,1/2,0],[0,1/4,0,1/2],[1/2,0,1,0],[0,1/2,0,1]],
 *   H = [[1,0,0,0],[0,1,0,0]], R = r I.
 * Per frame t, with the frame's points ordered by (y, x):
 *   1. every live track is predicted: s = F s, P = F P F^T + Q;
 *   2. every (track, point) pair with d2 = nu^T S^-1 nu <= gate is a candidate
 *      (nu = (x, y) - H s, S = H P H^T + R, S^-1 = adj(S) / det(S));
 *   3. candidates are taken in increasing (d2, track id, point index) order
 *      when neither side is taken yet (greedy nearest neighbour);
 *   4. a matched track is updated (K = P H^T S^-1, s += K nu,
 *      P = (I - K H) P); an unmatched one keeps its prediction and is dropped
 *      after more than max_miss missed frames in a row;
 *   5. every point left over starts a track: s = (x, y, 0, 0),
 *      P = diag(r, r, v0, v0), ids counting up from 0 in point order.
 * Double precision throughout, every matrix product summed over k = 0, 1, ...
 * from 0.0 without contraction, so the association and the states are
 * reproducible to the bit. */
enum {
    FZ_TRACK_MAX_TRACKS = 4096,              /* live tracks at once */
    FZ_TRACK_TOO_MANY_POINTS = 1,            /* a frame had more than 1024 points: the rest were ignored */
    FZ_TRACK_TOO_MANY_CANDIDATES = 2,        /* a frame had more than 2048 gated pairs: the rest were ignored */
    FZ_TRACK_TOO_MANY_TRACKS = 4             /* more than max_tracks live tracks: the newest were not started */
};

typedef struct fz_track_opts {
    double q;           /* process-noise intensity (pixels^2 per frame^4 of acceleration), >= 0 */
    double r;           /* measurement variance (pixels^2), > 0 */
    double gate;        /* candidate threshold on the squared Mahalanobis distance, >= 0 */
    double v0;          /* initial velocity variance of a new track (pixels^2 per frame^2), >= 0 */
    int32_t max_miss;   /* frames a track may go unmatched in a row before it is dropped, >= 0 */
    int32_t max_tracks; /* live tracks kept at once, 1 .. FZ_TRACK_MAX_TRACKS */
} fz_track_opts;

/* One live track after frame t. */
typedef struct fz_track {
    uint32_t t, id;
    int32_t status;     /* 0 predicted only, 1 updated by a point, 2 started by a point */
    uint32_t pad;
    double x, y, vx, vy;
} fz_track;

/* Defaults: q = 0.5, r = 1, gate = 9.21 (chi-square, 2 degrees of freedom,
 * 99%), v0 = 4, max_miss = 3, max_tracks = FZ_TRACK_MAX_TRACKS. */
fz_status fz_track_default_opts(fz_track_opts* out);
/* Device workspace fz_track_points needs for `frames` frames and a point
 * buffer of `point_capacity` records. */
size_t fz_track_workspace_bytes(int32_t frames, uint32_t point_capacity, const fz_track_opts* opts);
/* Track the points of a clip of `frames` frames:
 *   d_points, d_point_count, point_capacity: the chain's point buffer as
 *           fz_run_chain left it (device; min(*d_point_count, capacity)
 *           records are read; points with t >= frames are ignored);
 *   d_tracks, track_capacity: output records (device, caller-owned), one per
 *           live track and frame, in unspecified order;
 *   d_track_count: two device uint32: [0] the number of records (counting
 *           past the capacity), [1] FZ_TRACK_* flags of limits hit.
 * Asynchronous on `stream`; read the counts after it synchronises.
 * FZ_E_INVALID for bad sizes or options, FZ_E_WORKSPACE if ws_bytes is below
 * fz_track_workspace_bytes(). */
fz_status fz_track_points(const fz_point* d_points, const uint32_t* d_point_count, uint32_t point_capacity,
                          int32_t frames, const fz_track_opts* opts, fz_track* d_tracks, uint32_t* d_track_count,
                          uint32_t track_capacity, void* d_workspace, size_t ws_bytes, void* stream);

/* Message for the calling thread's last failed call ("" if none). */
const char* fz_last_error(void);

/* ---------------------------------------------------------------- cost model
 * The paper prices a candidate fused kernel by its predicted execution time
 * (Sec. VI, Fig. 5).  fz can learn that price: a 3-layer FP32 perceptron
 * F -> 64 -> 64 -> 1 (ReLU) maps the features of a group in one kernel
 * configuration to the natural log of its launch time in microseconds.  The
 * network is trained on the GPU with the calls below; fz_plan_chain with
 * FZ_COST_LEARNED evaluates it on the host for every group and kernel
 * configuration, keeps the fastest configuration per group, and partitions on
 * the predicted times.
 *
 * Parameters: one float array, row-major [out][in]:
 *   W1[64][F] b1[64] W2[64][64] b2[64] W3[64] b3[1]. */

/* Number of features of a group (the network's F). */
int32_t fz_cost_n_features(void);
/* Features of group i of a plan, as the learned planner computes them, into
 * out[0..cap); returns the count, or -1 on a bad argument. */
int32_t fz_plan_segment_features(const fz_plan* plan, int32_t i, float* out, int32_t cap);
/* Number of parameters for F features (F in [1, 32]), else -1. */
int32_t fz_mlp_param_count(int32_t n_features);
/* Device workspace of fz_mlp_loss_grad for n samples. */
size_t fz_mlp_workspace_bytes(int32_t n_features, int32_t n);
/* d_y[n] = network(d_x[n][F]) (device pointers).  Asynchronous on stream. */
fz_status fz_mlp_forward(const float* d_params, int32_t n_features, const float* d_x, int32_t n, float* d_y,
                         void* stream);
/* Loss L = mean((y - target)^2) over n samples into *d_loss and its gradient
 * with respect to every parameter into d_grad (device pointers; reductions in
 * a fixed order, so the result is deterministic). */
fz_status fz_mlp_loss_grad(const float* d_params, int32_t n_features, const float* d_x, const float* d_target,
                           int32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes, void* stream);
/* One Adam step (bias-corrected, step >= 1) on n_params parameters in place;
 * d_m and d_v are the caller's first and second moment buffers. */
fz_status fz_mlp_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t n_params,
                           int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Library version string. */
const char* fz_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FZ_H */
