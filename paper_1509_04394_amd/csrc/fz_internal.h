// Internal host-side declarations of the fz library.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fz.h"
#include "fz_ops.h"

namespace fz {

struct Segment {
    int first, last;        // stage indices of the user chain
    int cfirst, clast;      // the same in the compiled chain
    int tile;               // tile index (window groups), -1 for streaming groups
    int tile_w, tile_h;
    int tpb;                // frames per workgroup
    int halo, halo_t;
    int halo_y;             // halo along y (equal to halo except for generic groups with rx != ry)
    int lds_bytes;
    int streaming;
    int engine;             // FZ_ENGINE_TILE / ROW / STREAM
    int row_k, nstrips, nbands, nchunks;  // row-marching geometry
    int row_gen;            // 1: generic row kernel, 0: the Harris-chain kernel
    double bytes_per_px;
    double cost;
    int refused;            // a request this group's kernel cannot run (cost is +inf): 1 a band, 2 an IIR frame run
    int ckpt;               // generic groups: IIR states checkpointed per frame run (two launches, workspace)
};

struct Params {
    float sigma = 1.0f, k = 0.04f, thr = 1.0e8f;
    float gw[3] = {0, 0, 0};  // Gaussian weights w0, w1, w2 (FP32)
};

}  // namespace fz

struct fz_plan {
    std::vector<fz_stage> stages;
    int n = 0;
    int chain = 0, offset = 0;
    // generic chains (FZ_OP_STENCIL / BOX / POINT): chain = -1; the stencil
    // weights copied at plan time and each stage's first weight
    bool generic = false;
    std::vector<float> gweights;
    std::vector<int> gwoff;
    int W = 0, H = 0, T = 0;
    int lds_budget = 0;
    std::vector<double> cost;  // n x n, +inf where not allowed
    std::vector<fz::Segment> segs;
    double total = 0.0;
    fz::Params prm;
    bool has_nms = false;
    // requests the plan was made with (re-pricing for other clip sizes)
    int req_w = 0, req_h = 0, req_tpb = 0, req_engine = 0;
    // cached batch graph (hipGraph_t / hipGraphExec_t / hipStream_t) and its key
    void* batch_graph = nullptr;
    void* batch_exec = nullptr;
    void* capture_stream = nullptr;
    std::vector<uint64_t> batch_key;
    ~fz_plan();
};

namespace fz {

// thread-local error message
void set_error(const std::string& msg);
fz_status fail(fz_status code, const std::string& msg);

// Price of group [a..b] of plan p, with its tile / frames-per-block choice.
Segment price_group(const fz_plan& p, int a, int b, int tile_req_w, int tile_req_h, int tpb_req, int engine_req);

// Generic chains: price of group [a..b] (planner.cpp) and its launch (generic.hip)
Segment price_generic(const fz_plan& p, int a, int b, int req_w, int req_h, int req_tpb, int req_engine);
// Sec. VI-E, Eq. 6 box for a volume beta and halos dx (per side), dt (frames)
void eq6_box(double beta, double dx, double dt, double* x, double* t);
int launch_generic(const fz_plan& p, const Segment& g, const void* in, void* out, void* ckpt, void* stream);  // hipError_t
size_t ckpt_bytes(const fz_plan& p, const Segment& g);  // IIR checkpoints of group g (0 if none)
// Frame-boundary exchange of group g (a frame-difference row group; 0 otherwise).
size_t exchange_bytes(const fz_plan& p, const Segment& g);

// Learned prices (cost.cpp)
constexpr int COST_FEATURES = 20;
void group_features(const fz_plan& p, const Segment& g, float* f);
double mlp_predict(const float* prm, const float* x);
Segment price_group_learned(const fz_plan& p, int a, int b, const float* prm, int req_w, int req_h, int req_tpb,
                            int req_engine);

// Exact partition DP (Fig. 5 model) with the tie rule: fewer groups, then later cuts.
double partition_dp(const double* cost, int n, std::vector<int>& seg_last);

// Device side (run.hip)
fz_status run_plan(const fz_plan& p, const void* d_in, void* d_out, fz_point* d_points, uint32_t* d_count,
                   uint32_t cap, void* d_ws, size_t ws_bytes, void* stream);
size_t workspace_bytes(const fz_plan& p);

// Measured prices (measure.hip)
size_t measure_workspace_bytes(const fz_plan& p);
fz_status plan_measure(fz_plan& p, const void* d_in, void* ws, size_t ws_bytes, int reps, void* stream);

// The same partition re-priced for another video size (batch clips).
fz_plan* plan_for_size(const fz_plan& base, int W, int H, int T);
// Batch (batch.hip)
fz_status run_batch(fz_plan& p, const fz_clip* clips, int n, void* ws, size_t ws_bytes, void* stream);
size_t batch_workspace_bytes(const fz_plan& p, const fz_clip* clips, int n);
void release_batch(fz_plan& p);

// Generated kernels of generic groups (jit.cpp): source text, compile (no device needed), launch
std::string jit_source(const fz_plan& p, const Segment& g);
fz_status jit_prepare(const fz_plan& p, const Segment& g);
int launch_jit(const fz_plan& p, const Segment& g, const void* in, void* out, const void* ckpt,
               void* stream);  // hipError_t
int jit_load(const fz_plan& p, const Segment& g);  // hipError_t: compile and load on the current device

// Kalman tracking of feature points (track.hip)
size_t track_workspace_bytes(int T, uint32_t point_capacity, uint32_t max_tracks);
fz_status track_points(const fz_point* d_points, const uint32_t* d_count, uint32_t cap, int T, const fz_track_opts& o,
                       fz_track* d_tracks, uint32_t* d_track_count, uint32_t track_cap, void* ws, void* stream);

}  // namespace fz
