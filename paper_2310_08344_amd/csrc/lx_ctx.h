// The context behind the opaque lx_ctx handle (internal to the library).
#pragma once

#include <hip/hip_runtime_api.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "lx.h"
#include "lx_device.h"
#include "planner.h"

// A batch's device pipeline captured as a hipGraph: power iteration, the
// Newton coefficients and the first `launches` window launches, for one
// layout (key: sizes, launch shape and the workspace addresses the launches
// take).  Replayed by later calls with the same layout.
struct lx_batch_graph {
    std::vector<long long> key;
    hipGraphExec_t exec = nullptr;
    int launches = 0;
    unsigned long long last_use = 0;
};

// Workspaces of a batch of instances, grown on demand and kept.
struct lx_batch_ws {
    void* d_inst = nullptr;      // lx::BatchInst[n]
    void* d_ctl = nullptr;       // lx::LoopCtl[n]
    int* d_block_inst = nullptr; // instance of each workgroup
    double* d_coef = nullptr;    // n * ld Newton coefficients
    double* d_partials = nullptr;
    double* d_basis = nullptr;   // two basis vectors per instance
    unsigned* d_done = nullptr;  // instances that have finished
    void* h_inst = nullptr;      // pinned staging
    void* h_ctl = nullptr;
    int* h_block_inst = nullptr;
    unsigned* h_done = nullptr;  // [2] polled counters
    void* d_feat = nullptr;      // feature descriptors (lx_instance_features)
    void* h_feat = nullptr;
    size_t cap_d_inst = 0, cap_d_ctl = 0, cap_d_blk = 0, cap_coef = 0, cap_partials = 0, cap_basis = 0,
           cap_done = 0, cap_h_inst = 0, cap_h_ctl = 0, cap_h_blk = 0, cap_h_done = 0, cap_feat = 0;
    std::vector<lx_batch_graph> graphs;    // at most kBatchGraphs, least recently used replaced
    hipStream_t cap_stream = nullptr;      // private stream the graphs are captured on
    unsigned long long calls = 0;
    int use_graphs = 1;                    // lx_set_batch_graphs
    // tuned launch shapes per batch class (lx_tune_batched); key: any Burgers
    // instance, then the distinct sides
    std::map<std::vector<int>, lx::BatchShape> tuned;
};

struct lx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t n_max = 0;
    int k_max = 0;
    int timing = 0;
    // device workspaces
    double* ybuf[2] = {nullptr, nullptr};   // Newton basis ping-pong (FP64 or FP32 view)
    float* u32 = nullptr;                   // Burgers state in FP32 (FP32 sweeps)
    double* ws[3] = {nullptr, nullptr, nullptr};  // integrator stages (allocated on first use)
    std::vector<double*> sub_ws;            // substep workspaces (phi_i(tau A) v, two states)
    std::vector<double*> blk_ws;            // second buffer per output of speculative windows
    double* partials = nullptr;
    size_t partials_len = 0;
    lx::LoopCtl* ctl = nullptr;
    double* coef = nullptr;                 // k_max * kMaxPoints
    double* xi = nullptr;                   // kMaxPoints
    int xi_uploaded = 0;
    // pinned host staging
    lx::LoopCtl* h_ctl = nullptr;           // initial loop control (pinned)
    lx::SweepState* h_poll = nullptr;       // [2]: polled final-state slots (pinned)
    double* h_coef = nullptr;
    double* h_xi = nullptr;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> tev;            // timing events
    lx::NewtonSeries series[LX_K_MAX];      // per-output divided differences
    // launch shapes: forced by lx_set_tile, else tuned per (kind, nx, ny, K, prec)
    lx::Tile forced{0, 0, 0, 0, 0};         // tx == 0: not forced
    int depth_forced = 0;                   // lx_set_depth: 0 automatic, 1 or 2 iterations per launch
    int pair_th = 0, pair_nb = 0;           // lx_set_depth: forced leja_pair shape (0: automatic)
    int win_kind = 0;                       // lx_set_window_kernel: 0 automatic, 1 LDS tiles, 2 register march
    int win_bands = 0, win_nb = 0;          // lx_set_window_kernel: forced bands / workgroups (0: automatic)
    std::map<std::tuple<int, int, int, int, int>, lx::Tile> tuned;
    lx_batch_ws batch;
    std::vector<lx_predictor*> predictors;  // live predictors; lx_destroy frees them
    lx_stats stats{};
    std::string err;
};

// shared helpers of the C-ABI translation units (lx_api.cpp)
lx_status lx_internal_fail(lx_ctx* ctx, lx_status s, const char* fmt, ...);
lx_status lx_internal_check_op(lx_ctx* ctx, const lx_operator* op, size_t n_limit);
lx_status lx_internal_ensure_xi(lx_ctx* ctx, int M);
lx_status lx_internal_ensure_timing_events(lx_ctx* ctx, size_t n);
double lx_internal_elapsed(hipEvent_t a, hipEvent_t b);
void lx_internal_free_batch(lx_ctx* ctx);
