// C ABI of the Leja phi-action library (declarations and contracts in lx.h).
//
// Host side of the device-resident Leja loop: argument checks, the planner
// (Leja points; divided differences produced a chunk ahead of the sweeps
// that read them, while the GPU works), the initial loop state, then sweeps
// enqueued in chunks.  The sweeps decide by themselves when to stop (a
// converged loop turns later sweeps into no-ops); the host only looks at the
// state once per chunk, one chunk behind, to stop enqueuing: the launch that
// ends the loop writes the final state into pinned host memory, so looking
// costs an event wait and no copy.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "lx.h"
#include "lx_ctx.h"
#include "lx_device.h"
#include "planner.h"
#include "stencil_coeffs.h"

using lx::LoopCtl;
using lx::SweepState;
using lx::PowerArgs;
using lx::SweepArgs;
using lx::Tile;

namespace {

constexpr int kFirstChunk = 16;   // sweeps enqueued before the first look at the state
constexpr int kChunk = 8;         // sweeps per later chunk

lx_status fail(lx_ctx* ctx, lx_status s, const char* fmt, ...) {
    if (ctx != nullptr) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
        ctx->stats.status = s;
    }
    return s;
}

#define LX_HIP(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), LX_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                     \
    } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool is_diffadv(int kind) { return kind == LX_OP_DIFFADV2D || kind == LX_OP_DIFFADV2D_UP3; }

// the device kernels' operator code of an lx_op_kind
int opcode_of(int kind) {
    if (kind == LX_OP_DIFFADV2D) return lx::kOpDiffAdv;
    if (kind == LX_OP_DIFFADV2D_UP3) return lx::kOpDiffAdv3;
    return lx::kOpBurgersJ;
}

// the stencil of (A - c)/g as {E, W, N, S, C, E2, W2, N2, S2} for the
// diffusion-advection operators (second neighbours 0 for the five-point one)
void diffadv_stencil9(const lx_operator& op, double c, double g, double (&k9)[9]) {
    if (op.kind == LX_OP_DIFFADV2D_UP3) {
        lx::stencil_coeffs_up3(op.dx, op.dy, op.D, op.vx, op.vy, c, g, k9);
    } else {
        double k[5];
        lx::stencil_coeffs(0, op.dx, op.dy, op.D, op.vx, op.vy, op.nu, c, g, k);
        for (int i = 0; i < 9; ++i) k9[i] = i < 5 ? k[i] : 0.0;
    }
}

lx_status check_op(lx_ctx* ctx, const lx_operator* op) {
    if (op == nullptr) return fail(ctx, LX_EINVAL, "operator is NULL");
    if (op->kind != LX_OP_DIFFADV2D && op->kind != LX_OP_BURGERS2D && op->kind != LX_OP_DIFFADV2D_UP3)
        return fail(ctx, LX_EINVAL, "unknown operator kind %d", op->kind);
    if (op->nx < 3 || op->ny < 3) return fail(ctx, LX_EINVAL, "grid %dx%d: each side must be >= 3", op->nx, op->ny);
    if (op->kind == LX_OP_DIFFADV2D_UP3 && (op->nx < 4 || op->ny < 4))
        return fail(ctx, LX_EINVAL, "grid %dx%d: the third-order upwind operator needs sides >= 4", op->nx, op->ny);
    const size_t n = static_cast<size_t>(op->nx) * static_cast<size_t>(op->ny);
    if (n > ctx->n_max) return fail(ctx, LX_EINVAL, "grid of %zu points exceeds n_max %zu", n, ctx->n_max);
    if (!(op->dx > 0.0) || !(op->dy > 0.0) || !std::isfinite(op->dx) || !std::isfinite(op->dy))
        return fail(ctx, LX_EINVAL, "spacings must be finite and > 0");
    if (is_diffadv(op->kind) &&
        (!(op->D >= 0.0) || !std::isfinite(op->D) || !std::isfinite(op->vx) || !std::isfinite(op->vy)))
        return fail(ctx, LX_EINVAL, "diffusion-advection needs finite D >= 0 and finite v");
    if (op->kind == LX_OP_BURGERS2D && (!(op->nu >= 0.0) || !std::isfinite(op->nu)))
        return fail(ctx, LX_EINVAL, "Burgers needs finite nu >= 0");
    if (op->prec != LX_FP64 && op->prec != LX_FP32_SWEEP) return fail(ctx, LX_EINVAL, "unknown precision %d", op->prec);
    return LX_OK;
}

// Default launch shape (measured on MI355X with lx_tune at 1024^2..4096^2):
// two columns per lane when the rows allow 16-byte loads, 64 lanes along x
// when the grid is wide enough, one row per thread per tile, and 1024
// workgroups (4 per CU) looping over the tiles.
Tile choose_tile(int nx, int ny, bool vec2_ok) {
    (void)ny;
    Tile t;
    t.vec = (vec2_ok && nx % 2 == 0) ? 2 : 1;
    int tx = 64;
    while (tx > 4 && tx * t.vec > nx) tx >>= 1;
    t.tx = tx;
    t.ty = lx::kBlockThreads / tx;
    t.ry = 1;
    t.nb = 1024;
    return t;
}

int tiles_of(const Tile& t, int nx, int ny) {
    return ((nx + t.cols() - 1) / t.cols()) * ((ny + t.rows() - 1) / t.rows());
}

// workgroups in the grid: the shape's choice (0 = one per tile), at most one
// per tile, a multiple of 8 once there are at least 8 (one band per XCD)
int grid_size(const Tile& t, int tiles) {
    int nb = (t.nb <= 0 || t.nb > tiles) ? tiles : t.nb;
    if (nb >= 8) nb &= ~7;
    return std::max(nb, 1);
}

lx_status ensure_xi(lx_ctx* ctx, int M) {
    if (M <= ctx->xi_uploaded) return LX_OK;
    if (!lx::leja_points(M, ctx->h_xi)) return fail(ctx, LX_EINVAL, "cannot build %d Leja points", M);
    LX_HIP(ctx, hipMemcpyAsync(ctx->xi, ctx->h_xi, sizeof(double) * M, hipMemcpyHostToDevice, ctx->stream));
    LX_HIP(ctx, hipStreamSynchronize(ctx->stream));   // h_xi is reused by the next extension
    ctx->xi_uploaded = M;
    return LX_OK;
}

lx_status ensure_timing_events(lx_ctx* ctx, size_t n) {
    while (ctx->tev.size() < n) {
        hipEvent_t e;
        LX_HIP(ctx, hipEventCreate(&e));
        ctx->tev.push_back(e);
    }
    return LX_OK;
}

lx_status ensure_partials(lx_ctx* ctx, size_t need) {
    if (need <= ctx->partials_len) return LX_OK;
    LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->partials);
    ctx->partials = nullptr;
    ctx->partials_len = 0;
    if (hipMalloc(&ctx->partials, sizeof(double) * need) != hipSuccess)
        return fail(ctx, LX_ENOMEM, "partials workspace of %zu doubles", need);
    ctx->partials_len = need;
    return LX_OK;
}

bool valid_tile(const Tile& t) {
    const bool ry_ok = t.ry == 1 || t.ry == 2 || t.ry == 4 || t.ry == 8;
    return t.tx >= 1 && t.ty >= 1 && t.tx * t.ty == lx::kBlockThreads && ry_ok && (t.vec == 1 || t.vec == 2) &&
           t.nb >= 0;
}

// forced shape, else the tuned one, else the built-in rule
Tile pick_tile(const lx_ctx* ctx, const lx_operator& op, int K, bool vec2_ok) {
    Tile t;
    if (ctx->forced.tx != 0) {
        t = ctx->forced;
    } else {
        auto it = ctx->tuned.find(std::make_tuple(op.kind, op.nx, op.ny, K, op.prec));
        t = (it != ctx->tuned.end()) ? it->second : choose_tile(op.nx, op.ny, vec2_ok);
    }
    if (t.vec == 2 && !(vec2_ok && op.nx % 2 == 0)) t.vec = 1;
    return t;
}

void set_stencil(SweepArgs& a, const lx_operator& op, double c, double g) {
    if (is_diffadv(op.kind)) {
        double k[9];
        diffadv_stencil9(op, c, g, k);
        a.aE = k[0];
        a.aW = k[1];
        a.aN = k[2];
        a.aS = k[3];
        a.aC = k[4];
        a.aE2 = k[5];
        a.aW2 = k[6];
        a.aN2 = k[7];
        a.aS2 = k[8];
    } else {
        double k[5];
        lx::stencil_coeffs(1, op.dx, op.dy, op.D, op.vx, op.vy, op.nu, c, g, k);
        a.kx = k[0];
        a.ky = k[1];
        a.gx = k[2];
        a.gy = k[3];
        a.kC = k[4];
    }
}

void load_tune_cache(lx_ctx* ctx) {
    const char* path = std::getenv("LX_TUNE_CACHE");
    if (path == nullptr || *path == 0) return;
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f) != nullptr) {
        int kind, nx, ny, K, prec;
        Tile t;
        if (std::sscanf(line, "{\"kind\": %d, \"nx\": %d, \"ny\": %d, \"K\": %d, \"prec\": %d, \"tx\": %d, "
                              "\"ty\": %d, \"ry\": %d, \"vec\": %d, \"nb\": %d, \"depth\": %d, \"th\": %d, "
                              "\"pnb\": %d, \"stream\": %d, \"bands\": %d, \"snb\": %d",
                        &kind, &nx, &ny, &K, &prec, &t.tx, &t.ty, &t.ry, &t.vec, &t.nb, &t.depth, &t.th, &t.pnb,
                        &t.stream, &t.bands, &t.snb) == 16 &&
            valid_tile(t) && t.depth >= 1 && t.depth <= 8 && t.depth != 5 && t.depth != 7 &&
            (t.th == 8 || t.th == 16 || t.th == 32) && t.pnb >= 0 && (t.stream == 0 || t.stream == 1) &&
            t.bands >= 0 && t.snb >= 0) {
            ctx->tuned[std::make_tuple(kind, nx, ny, K, prec)] = t;
            continue;
        }
        // a batch class's shape (lx_tune_batched): {"batch_class": [b, nx, ny, ...], "depth": d, "th": t, "ppw": p
        const char* q = std::strstr(line, "{\"batch_class\": [");
        if (q != line) continue;
        q += std::strlen("{\"batch_class\": [");
        std::vector<int> cls;
        char* end = nullptr;
        for (;;) {
            const long v = std::strtol(q, &end, 10);
            if (end == q) break;
            cls.push_back(static_cast<int>(v));
            q = end;
            while (*q == ',' || *q == ' ') ++q;
        }
        lx::BatchShape b;
        if (*q == ']' && cls.size() >= 3 && cls.size() % 2 == 1 &&
            std::sscanf(q, "], \"depth\": %d, \"th\": %d, \"ppw\": %d", &b.depth, &b.th, &b.ppw) == 3 &&
            (b.depth == 1 || b.depth == 2 || b.depth == lx::kBatchBlockDepth) && (b.th == 8 || b.th == 16) &&
            b.ppw > 0 && b.ppw <= (1 << 22))
            ctx->batch.tuned[cls] = b;
    }
    std::fclose(f);
}

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return static_cast<double>(ms);
}

struct LejaCall {
    const lx_operator* op;
    const double* u;
    const double* v;
    int K;
    int l[LX_K_MAX];
    double alpha[LX_K_MAX];
    double sigma[LX_K_MAX];
    double* out[LX_K_MAX];
    double h, c, gamma;
    lx_leja_opts o;
    // lx_phi_leja_static: the library's static device scratch, which then
    // holds the basis pair, the windows' second output buffers and the
    // partial sums (nothing is allocated); nullptr: the context's workspaces
    double* scratch = nullptr;
};

// Whether a call may run its windows by register marching at this depth
// (the five-point operators, FP64 or FP32 sweeps).
bool stream_ok(const lx_operator& op, int K, int depth) {
    if (op.kind != LX_OP_DIFFADV2D && op.kind != LX_OP_BURGERS2D) return false;
    // vectors of at most 2^30 bytes (the kernel's buffer offsets)
    return op.nx % 2 == 0 && op.nx >= depth && op.ny >= depth &&
           static_cast<long>(op.nx) * op.ny * 8 <= (1L << 30) &&
           lx::stream_has(opcode_of(op.kind), K, depth, op.prec == LX_FP32_SWEEP);
}

// Iterations per launch for this call: forced by lx_set_depth, else the
// tuned entry's, else two.  Two or more need FP64 sweeps and 16-byte pairs;
// windows of three or more need sides of depth x radius cells (else two),
// and six the five-point diffusion-advection operator (else four).
void choose_depth(const lx_ctx* ctx, const lx_operator& op, int K, bool vec2_ok, Tile& t) {
    const bool pair_ok = op.prec == LX_FP64 && vec2_ok && op.nx % 2 == 0;
    // register-marching windows also take FP32 sweeps
    const bool march_ok = vec2_ok && op.nx % 2 == 0;
    auto it = ctx->tuned.find(std::make_tuple(op.kind, op.nx, op.ny, K, op.prec));
    int depth = 2;
    if (ctx->depth_forced != 0) depth = ctx->depth_forced;
    else if (it != ctx->tuned.end()) depth = it->second.depth;
    // windows stage a halo of depth * radius cells, which the periodic index
    // wrap allows only on sides of at least that many cells
    // windows by register marching: forced by lx_set_window_kernel, else the
    // tuned entry's choice; eight iterations only that way
    const bool tuned_stream = it != ctx->tuned.end() && it->second.stream && it->second.depth == depth;
    t.stream = 0;
    if (march_ok && depth >= 3 && (ctx->win_kind == 2 || (ctx->win_kind == 0 && tuned_stream)) &&
        stream_ok(op, K, depth)) {
        t.stream = 1;
        t.depth = depth;
        t.bands = ctx->win_bands != 0 ? ctx->win_bands : (tuned_stream ? it->second.bands : 0);
        t.snb = ctx->win_nb != 0 ? ctx->win_nb : (tuned_stream ? it->second.snb : 0);
        return;
    }
    if (depth == 8) depth = 6;
    const int halo = depth * (op.kind == LX_OP_DIFFADV2D_UP3 ? 2 : 1);
    if (depth >= 3 && (op.nx < halo || op.ny < halo)) depth = 2;
    if (depth == 6 && op.kind != LX_OP_DIFFADV2D) depth = 4;   // six: the five-point operator only
    t.depth = (depth >= 2 && pair_ok) ? depth : 1;
    if (it != ctx->tuned.end() && it->second.depth >= 2 && it->second.depth == t.depth && !it->second.stream) {
        t.th = it->second.th;
        t.pnb = it->second.pnb;
    } else {
        t.th = 16;
        t.pnb = 1024;
    }
    if (ctx->pair_th != 0) t.th = ctx->pair_th;
    if (ctx->pair_nb != 0) t.pnb = ctx->pair_nb;
    // a radius-2 stencil stages 8 edge cells per row, and three or four
    // iterations per launch hold two levels in LDS: tiles of at most 16 rows
    if ((op.kind == LX_OP_DIFFADV2D_UP3 || t.depth >= 3) && t.th > 16) t.th = 16;
}

lx_status ensure_blk_ws(lx_ctx* ctx, int K) {
    while (static_cast<int>(ctx->blk_ws.size()) < K) {
        double* p = nullptr;
        if (hipMalloc(&p, sizeof(double) * ctx->n_max) != hipSuccess)
            return fail(ctx, LX_ENOMEM, "second output buffers of the multi-iteration loop");
        ctx->blk_ws.push_back(p);
    }
    return LX_OK;
}

// workgroups of a leja_pair grid: at most one per tile, a multiple of 8 once
// there are at least 8
int pair_grid(int pnb, int tiles) {
    int nb = (pnb <= 0 || pnb > tiles) ? tiles : pnb;
    if (nb >= 8) nb &= ~7;
    return std::max(nb, 1);
}

// Grid of a register-marching launch (leja_stream, power_stream): strips of
// at most 128 - 2D output columns (stream_strips) by bands of rows, one item
// per wavefront.  By default the bands make one resident round of wavefronts
// (no partial second round), with bands of at least 4D rows so that the D
// rows staged above and below a band stay a small share of it; workgroups
// are a multiple of 8 when that stays within one round (each XCD then takes
// a contiguous run of bands).
struct StreamGrid {
    int strips, bands, nb;
};

StreamGrid stream_grid(int op, bool fp32, int nx, int ny, int K, int D, int bands, int nb, bool power) {
    StreamGrid g;
    g.strips = lx::stream_strips(nx, D);
    const int resident = lx::stream_resident(op, K, D, fp32, power ? 1 : 0);
    const int waves = (resident > 0 ? resident : 512) * (lx::kBlockThreads / 64);
    int by = bands;
    if (by <= 0) by = std::max(1, std::min(waves / g.strips, ny / (4 * D)));
    g.bands = std::max(1, std::min(by, ny));
    const int items = g.strips * g.bands;
    int wgs = nb > 0 ? nb : (items + 3) / 4;
    if (nb <= 0 && resident > 0) wgs = std::min(wgs, resident);
    if (nb <= 0 && wgs >= 8) {
        const int up = (wgs + 7) & ~7;
        if (resident <= 0 || up <= resident) wgs = up;
    }
    g.nb = std::max(wgs, 1);
    return g;
}

// The device-resident Newton-Leja loop (Sec. 2.1, Eq. (2); stop rule of
// Sec. 2.2), one or more iterations per launch.  Fills ctx->stats.
lx_status run_leja(lx_ctx* ctx, const LejaCall& q) {
    const lx_operator& op = *q.op;
    const int nx = op.nx, ny = op.ny;
    const long N = static_cast<long>(nx) * ny;
    const int K = q.K;
    const int M = q.o.max_iters + 1;
    const bool fp32 = op.prec == LX_FP32_SWEEP;
    lx_stats& S = ctx->stats;
    S = lx_stats{};
    const bool timing = ctx->timing != 0 && q.scratch == nullptr;

    bool vec2 = aligned16(q.v) && (q.u == nullptr || aligned16(q.u));
    for (int k = 0; k < K; ++k) vec2 = vec2 && aligned16(q.out[k]);
    Tile t = pick_tile(ctx, op, K, vec2);
    choose_depth(ctx, op, K, vec2, t);
    const bool pair = t.depth == 2;
    const bool blk = t.depth >= 3;          // speculative windows of D iterations
    const int D = t.depth;
    // coefficients the loop may read: d_0..d_{NC-1} (a two-iteration launch
    // also forms the norm its last, deferred term would give; a window that
    // starts below max_iters reads up to D terms on)
    const int NC = blk ? M + D : (pair ? M + 1 : M);

    // ---- planner: Leja points now, Newton coefficients chunk by chunk ----
    const auto t0 = std::chrono::steady_clock::now();
    lx_status s = ensure_xi(ctx, NC);
    if (s != LX_OK) return s;
    for (int k = 0; k < K; ++k)
        ctx->series[k].reset(q.l[k], q.alpha[k], q.sigma[k], q.h, q.c, q.gamma, ctx->h_xi);
    int have = 0;          // coefficients d_0..d_{have-1} computed and enqueued for upload
    double plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // the launch that ends the loop writes its final state here (pinned)
    volatile SweepState* pub = ctx->h_poll;
    pub->done = 0;
    // stop_on_done: a look ahead, abandoned (nothing uploaded, *ended set)
    // once the loop has published its final state; the series then no longer
    // match `have`, and the caller ends the loop
    auto ensure_coeffs = [&](int upto, bool* ended = nullptr) -> lx_status {
        upto = std::min(upto, NC);
        if (upto <= have) return LX_OK;
        const auto ta = std::chrono::steady_clock::now();
        for (int j = have; j < upto; ++j) {
            if (ended != nullptr && pub->done) {
                *ended = true;
                plan_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
                return LX_OK;
            }
            for (int k = 0; k < K; ++k) ctx->h_coef[static_cast<size_t>(k) * NC + j] = ctx->series[k].next();
        }
        // one copy for all outputs (each copy is a launch on the stream): the
        // span from d_have of output 0 to d_{upto-1} of output K-1 also
        // carries the coefficients already on the device (the same values)
        // and slots past upto that no launch reads before a later copy
        // brings their final values
        const size_t off = static_cast<size_t>(have);
        const size_t len = static_cast<size_t>(K - 1) * NC + upto - have;
        LX_HIP(ctx, hipMemcpyAsync(ctx->coef + off, ctx->h_coef + off, sizeof(double) * len, hipMemcpyHostToDevice,
                                   ctx->stream));
        have = upto;
        plan_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
        return LX_OK;
    };

    LoopCtl& init = *ctx->h_ctl;
    std::memset(&init, 0, sizeof(init));
    init.rtol = q.o.rtol;
    init.atol = q.o.atol;
    init.fp32_switch = fp32 ? q.o.fp32_switch : -1.0;
    init.max_iters = q.o.max_iters;
    SweepState& s0 = init.slot[0];
    s0.out32 = (fp32 && q.o.fp32_switch == 0.0) ? 1 : 0;
    for (int k = 0; k < K; ++k) {
        s0.active[k] = 1;
        s0.iters[k] = q.o.max_iters;
    }
    LX_HIP(ctx, hipMemcpyAsync(ctx->ctl, &init, sizeof(LoopCtl), hipMemcpyHostToDevice, ctx->stream));

    if (fp32 && op.kind == LX_OP_BURGERS2D) LX_HIP(ctx, lx::launch_to_fp32(q.u, ctx->u32, N, ctx->stream));

    // ---- sweep arguments ----
    SweepArgs a{};
    a.nx = nx;
    a.ny = ny;
    if (t.stream) {
        const StreamGrid g = stream_grid(opcode_of(op.kind), fp32, nx, ny, K, D, t.bands, t.snb, false);
        a.tiles_x = g.strips;
        a.tiles_y = g.bands;
        a.nb = g.nb;
    } else if (pair || blk) {
        a.tiles_x = (nx + 127) / 128;
        a.tiles_y = (ny + t.th - 1) / t.th;
        a.nb = pair_grid(t.pnb, a.tiles_x * a.tiles_y);
    } else {
        a.tiles_x = (nx + t.cols() - 1) / t.cols();
        a.tiles_y = (ny + t.rows() - 1) / t.rows();
        a.nb = grid_size(t, a.tiles_x * a.tiles_y);
    }
    a.ld = NC;
    set_stencil(a, op, q.c, q.gamma);
    a.inv_sqrtN = 1.0 / std::sqrt(static_cast<double>(N));
    a.v = q.v;
    a.ybuf[0] = q.scratch != nullptr ? q.scratch : ctx->ybuf[0];
    a.ybuf[1] = q.scratch != nullptr ? q.scratch + lx::kStaticPoints : ctx->ybuf[1];
    a.u = q.u;
    a.u32 = ctx->u32;
    for (int k = 0; k < K; ++k) a.p[k] = q.out[k];
    if (blk && q.scratch != nullptr) {
        for (int k = 0; k < K; ++k) a.p2[k] = q.scratch + (2 + k) * lx::kStaticPoints;
    } else if (blk) {
        s = ensure_blk_ws(ctx, K);
        if (s != LX_OK) return s;
        for (int k = 0; k < K; ++k) a.p2[k] = ctx->blk_ws[k];
    }
    a.coef = ctx->coef;
    a.xi = ctx->xi;
    a.ctl = ctx->ctl;
    a.pub = ctx->h_poll;
    const int opcode = opcode_of(op.kind);
    const size_t need_partials = 2 * static_cast<size_t>(a.nb) * (1 + K) * (blk ? D : (pair ? 2 : 1));
    if (q.scratch != nullptr) {
        if (need_partials > lx::kStaticPartials)
            return fail(ctx, LX_EINVAL, "launch shape needs %zu partial sums, the static scratch holds %zu",
                        need_partials, lx::kStaticPartials);
        a.partials = q.scratch + (2 + lx::kKMax) * lx::kStaticPoints;
    } else {
        s = ensure_partials(ctx, need_partials);
        if (s != LX_OK) return s;
        a.partials = ctx->partials;
    }

    // ---- chunked, device-resident loop ----
    // single: launch m (0 <= m < max_iters) is sweep m, which reads d_m (its
    // stop decision) and d_{m+1}; launch max_iters only takes the last
    // decision.  pair: launch L takes the decisions at terms 2L-1 and 2L and
    // then sweeps 2L and 2L+1; by launch ceil(max_iters/2) the loop has
    // ended, and the launch after it publishes a flush's final state.
    // blk: windows start below max_iters (at most ceil(max_iters/D) of
    // them), each stop event re-executes one (at most K), and one launch
    // after the last publishes the final state.
    const int max_iters = q.o.max_iters;
    const int last = blk ? (max_iters + D - 1) / D + K + 2
                         : (pair ? (max_iters + 1) / 2 + 1 : max_iters);   // last launch index
    const int per = blk ? D : (pair ? 2 : 1);                               // iterations per launch
    if (timing) {
        s = ensure_timing_events(ctx, static_cast<size_t>(last) + 2);
        if (s != LX_OK) return s;
        LX_HIP(ctx, hipEventRecord(ctx->tev[0], ctx->stream));
    }
    auto coeffs_for = [&](int launches) { return per * launches + 1; };   // d_0 .. d_{per*launches}
    int launched = 0, chunk_id = 0, last_slot = -1;
    // launches per chunk: about kFirstChunk and kChunk iterations, but at
    // least three and two launches, so that the queue never runs dry while
    // the host looks at the state of the chunk before.  A window is long
    // enough on its own to hide the host's work on the next chunk's
    // coefficients, so windows start with one launch: the GPU waits only for
    // d_0..d_D, not for the first three windows' coefficients (the first
    // look still comes after three launches).
    const int first_chunk = blk ? 1 : std::max(3, kFirstChunk / per), next_chunk = std::max(2, kChunk / per);
    int chunk = first_chunk;
    bool seen_done = false;   // a look at the state found the final one
    while (launched <= last) {
        const int n = std::min(chunk, last + 1 - launched);
        s = ensure_coeffs(coeffs_for(launched + n));
        if (s != LX_OK) return s;
        for (int i = 0; i < n; ++i) {
            const int L = launched + i;
            if (t.stream) LX_HIP(ctx, lx::launch_leja_stream(opcode, K, D, fp32, a, L, ctx->stream));
            else if (blk) LX_HIP(ctx, lx::launch_leja_block(opcode, K, t.th, D, a, L, ctx->stream));
            else if (pair) LX_HIP(ctx, lx::launch_leja_pair(opcode, K, t.th, a, L, ctx->stream));
            else LX_HIP(ctx, lx::launch_leja_sweep(opcode, K, fp32, t, a, L, ctx->stream));
            if (timing && L < last) LX_HIP(ctx, hipEventRecord(ctx->tev[L + 1], ctx->stream));
        }
        launched += n;
        const int slot = chunk_id & 1;
        LX_HIP(ctx, hipEventRecord(ctx->poll_ev[slot], ctx->stream));
        last_slot = slot;
        if (chunk_id >= 1) {
            // the next chunk's coefficients are prepared while the GPU works,
            // unless the final state appears meanwhile (the host then returns
            // at once instead of finishing them first)
            s = ensure_coeffs(coeffs_for(std::min(launched + next_chunk, last)), &seen_done);
            if (s != LX_OK) return s;
            // the chunk before has run: has a launch published the final state?
            if (!seen_done && !pub->done) LX_HIP(ctx, hipEventSynchronize(ctx->poll_ev[slot ^ 1]));
            if (seen_done || pub->done) {
                seen_done = true;
                break;
            }
        }
        ++chunk_id;
        chunk = next_chunk;
    }
    // Once the final state is published, every launch that writes an output
    // has finished (they precede the publishing launch on the stream); the
    // launches still queued only read the loop state and return, so the call
    // does not wait for them.
    if (!seen_done) LX_HIP(ctx, hipEventSynchronize(ctx->poll_ev[last_slot]));
    // the device writes `done` after the rest of the state (both at system
    // scope): what follows a read of done = 1 sees the whole state
    std::atomic_thread_fence(std::memory_order_acquire);
    const SweepState fin = *const_cast<const SweepState*>(ctx->h_poll);
    if (!fin.done) return fail(ctx, LX_EDEVICE, "the device loop did not record a final state");

    S.n_fp32 = fin.n_fp32;
    for (int k = 0; k < K; ++k) {
        S.iters[k] = fin.iters[k];
        S.err[k] = fin.err[k];
        S.pnorm[k] = fin.pnorm[k];
    }
    // algorithmic bytes of the launches that did work
    double bytes = 0.0;
    const double ub = op.kind == LX_OP_BURGERS2D ? 8.0 : 0.0;
    if (blk) {
        // counted on the device by the launches that did work (windows and
        // their re-executions): y in and out, and per output taking terms a
        // read and a write of p (the first window writes p without reading it)
        S.n_launch = fin.n_work;
        S.n_apply = fin.n_levels;
        bytes = fin.bytes_pp * static_cast<double>(N);
    } else if (!pair) {
        // per sweep: the basis read and write, the Burgers state read, and per
        // unconverged output a read and a write of p (sweep 0 writes
        // p_1 = d_0 v + d_1 y_1 without reading it)
        S.n_apply = fin.iter;
        S.n_launch = fin.iter;
        for (int m = 0; m < fin.iter; ++m) {
            const bool w32 = m >= fin.iter - fin.n_fp32;
            const bool r32 = m >= 1 && (m - 1) >= fin.iter - fin.n_fp32;
            double b = (r32 ? 4.0 : 8.0) + (w32 ? 4.0 : 8.0);
            if (op.kind == LX_OP_BURGERS2D) b += w32 ? 4.0 : 8.0;
            for (int k = 0; k < K; ++k) {
                if (m < fin.iters[k]) b += (m == 0) ? 8.0 : 16.0;
            }
            bytes += b * static_cast<double>(N);
        }
    } else {
        // the loop ended at the test of term T: launches 0..F-1 ran both
        // sweeps, and an even T left a deferred term for one more launch.
        // Per two-sweep launch: y_m in, y_{m+2} out, the Burgers state, and
        // per output still taking terms a read and a write of p (launch 0
        // writes p without reading it).
        const int T = fin.iter;
        const int F = (T + 1) / 2;
        const bool flush = T % 2 == 0;
        S.n_apply = 2 * F;
        S.n_launch = F + (flush ? 1 : 0);
        for (int L = 0; L < F; ++L) {
            double b = 16.0 + ub;
            for (int k = 0; k < K; ++k) {
                if (L == 0) b += 8.0;
                else if (fin.iters[k] >= 2 * L) b += 16.0;
            }
            bytes += b * static_cast<double>(N);
        }
        if (flush) {
            double b = 8.0;
            for (int k = 0; k < K; ++k)
                if (fin.iters[k] >= T) b += 16.0;
            bytes += b * static_cast<double>(N);
        }
    }
    S.depth = per;
    S.marching = t.stream ? 1 : 0;
    S.bytes = bytes;
    S.plan_ms = plan_ms;
    if (timing && S.n_launch > 0) {
        // events follow every launch: a launch's interval also holds the stop
        // decision the next one takes first (a few microseconds); the last
        // working launch's event precedes the final state on the stream
        LX_HIP(ctx, hipEventSynchronize(ctx->tev[S.n_launch]));
        S.first_sweep_ms = elapsed(ctx->tev[0], ctx->tev[1]);
        S.loop_ms = elapsed(ctx->tev[0], ctx->tev[S.n_launch]);
        S.sweep_ms = S.loop_ms;
    }
    S.status = fin.status;
    if (S.status == LX_ENONFINITE) return fail(ctx, LX_ENONFINITE, "a norm became NaN or Inf at sweep %d", fin.iter);
    if (S.status == LX_ENOTCONV) {
        ctx->err = "not converged within max_iters";
        return LX_ENOTCONV;
    }
    return LX_OK;
}

lx_status check_leja_opts(lx_ctx* ctx, const lx_leja_opts* o, lx_leja_opts* out) {
    lx_leja_opts d{1e-8, 0.0, 500, 1e4, 0};
    if (o != nullptr) d = *o;
    if (!(d.rtol >= 0.0) || !(d.atol >= 0.0) || !std::isfinite(d.rtol) || !std::isfinite(d.atol))
        return fail(ctx, LX_EINVAL, "tolerances must be finite and >= 0");
    if (d.max_iters < 1 || d.max_iters > LX_MAX_ITERS)
        return fail(ctx, LX_EINVAL, "max_iters %d outside 1..%d", d.max_iters, LX_MAX_ITERS);
    if (!(d.fp32_switch >= 0.0)) return fail(ctx, LX_EINVAL, "fp32_switch must be >= 0");
    if (d.substeps < 0 || d.substeps > LX_MAX_SUBSTEPS)
        return fail(ctx, LX_EINVAL, "substeps %d outside 0..%d", d.substeps, LX_MAX_SUBSTEPS);
    *out = d;
    return LX_OK;
}

lx_status check_shift(lx_ctx* ctx, double h, double c, double gamma) {
    if (!(h > 0.0) || !std::isfinite(h)) return fail(ctx, LX_EINVAL, "step h must be finite and > 0");
    if (!(c <= 0.0) || !std::isfinite(c)) return fail(ctx, LX_EINVAL, "shift c must be finite and <= 0");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(ctx, LX_EINVAL, "scale gamma must be finite and > 0");
    return LX_OK;
}

// Largest alpha*h*gamma of one Leja call under automatic substeps: half of
// the largest value at which the plain loop was still seen to converge.
constexpr double kSubstepHGamma = 300.0;

// rms norm (l2 / sqrt(N)) of a device vector: per-workgroup sums of squares
// (the power iteration's norm kernel), added on the host in workgroup order
lx_status rms_norm(lx_ctx* ctx, const double* x, long N, double* out) {
    constexpr int nb = 256;
    lx_status s = ensure_partials(ctx, 2 * nb);
    if (s != LX_OK) return s;
    double h[nb];
    LX_HIP(ctx, lx::launch_power_norm(x, N, nb, ctx->partials, ctx->stream));
    LX_HIP(ctx, hipMemcpyAsync(h, ctx->partials + nb, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double t = 0.0;
    for (double v : h) t += v;
    *out = std::sqrt(t / static_cast<double>(N));
    return LX_OK;
}

lx_status ensure_sub_ws(lx_ctx* ctx, size_t count) {
    while (ctx->sub_ws.size() < count) {
        double* p = nullptr;
        if (hipMalloc(&p, sizeof(double) * ctx->n_max) != hipSuccess)
            return fail(ctx, LX_ENOMEM, "substep workspace allocation failed");
        ctx->sub_ws.push_back(p);
    }
    return LX_OK;
}

// The Leja call with substeps (lx_leja_opts.substeps): every output over s
// substeps of tau = alpha h / s.  exp: s exp actions in a row, sigma on the
// last.  l >= 1: phi-function time stepping on u(t) = t^l phi_l(tA) v,
//   u(tau) = tau^l phi_l(tau A) v,
//   u(t + tau) = e^{tau A} u(t) + sum_{i=1..l} tau^i t^{l-i}/(l-i)! phi_i(tau A) v,
//   out = sigma u(alpha h) / (alpha h)^l,
// with phi_1..phi_L(tau A) v for all outputs of one alpha from vertical
// calls of at most k_max outputs.  Fills ctx->stats with the sums.
lx_status run_leja_sub(lx_ctx* ctx, const LejaCall& q) {
    double amax = 0.0;
    for (int k = 0; k < q.K; ++k) amax = std::max(amax, q.alpha[k]);
    int s = q.o.substeps;
    if (s == 0) {
        const double want = std::ceil(amax * q.h * q.gamma / kSubstepHGamma);
        s = static_cast<int>(std::min<double>(std::max(1.0, want), LX_MAX_SUBSTEPS));
    }
    if (s <= 1) {
        const lx_status st = run_leja(ctx, q);
        ctx->stats.substeps = 1;
        return st;
    }
    const long N = static_cast<long>(q.op->nx) * q.op->ny;
    lx_stats acc{};
    int iters[LX_K_MAX] = {0, 0, 0, 0};
    double errs[LX_K_MAX] = {0, 0, 0, 0};
    lx_status worst = LX_OK;
    // one Leja call, its statistics added; LX_ENOTCONV is remembered
    auto call = [&](const LejaCall& c) -> lx_status {
        const lx_status st = run_leja(ctx, c);
        const lx_stats& t = ctx->stats;
        acc.n_apply += t.n_apply;
        acc.n_fp32 += t.n_fp32;
        acc.n_launch += t.n_launch;
        acc.plan_ms += t.plan_ms;
        acc.loop_ms += t.loop_ms;
        acc.sweep_ms += t.sweep_ms;
        acc.bytes += t.bytes;
        acc.depth = t.depth;
        acc.marching = t.marching;
        if (st == LX_ENOTCONV) {
            worst = LX_ENOTCONV;
            return LX_OK;
        }
        return st;
    };
    auto single = [&](const double* v, double* out, int l, double tau, double sigma) {
        LejaCall c = q;
        c.v = v;
        c.K = 1;
        c.l[0] = l;
        c.alpha[0] = 1.0;
        c.sigma[0] = sigma;
        c.out[0] = out;
        c.h = tau;
        return c;
    };
    bool done[LX_K_MAX] = {false, false, false, false};
    for (int k0 = 0; k0 < q.K; ++k0) {
        if (done[k0]) continue;
        const double alpha = q.alpha[k0];
        const double H = alpha * q.h, tau = H / s;
        int L = 0;
        for (int k = k0; k < q.K; ++k)
            if (q.alpha[k] == alpha) L = std::max(L, q.l[k]);
        lx_status st = ensure_sub_ws(ctx, static_cast<size_t>(L) + 2);
        if (st != LX_OK) return st;
        double* const* P = ctx->sub_ws.data();            // P[i-1] = phi_i(tau A) v
        double* A = ctx->sub_ws[L];
        double* B = ctx->sub_ws[L + 1];
        int piters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i0 = 1; i0 <= L; i0 += ctx->k_max) {
            LejaCall c = q;
            c.K = std::min(ctx->k_max, L - i0 + 1);
            c.h = tau;
            for (int j = 0; j < c.K; ++j) {
                c.l[j] = i0 + j;
                c.alpha[j] = 1.0;
                c.sigma[j] = 1.0;
                c.out[j] = P[i0 + j - 1];
            }
            st = call(c);
            if (st != LX_OK) return st;
            for (int j = 0; j < c.K; ++j) piters[i0 + j - 1] = ctx->stats.iters[j];
        }
        for (int k = k0; k < q.K; ++k) {
            if (q.alpha[k] != alpha) continue;
            done[k] = true;
            const int l = q.l[k];
            if (l == 0) {
                const double* cur = q.v;
                for (int j = 0; j < s; ++j) {
                    double* dst = (j == s - 1) ? q.out[k] : ((j & 1) ? B : A);
                    st = call(single(cur, dst, 0, tau, j == s - 1 ? q.sigma[k] : 1.0));
                    if (st != LX_OK) return st;
                    iters[k] += ctx->stats.iters[0];
                    errs[k] = ctx->stats.err[0];
                    cur = dst;
                }
                continue;
            }
            iters[k] = piters[l - 1];
            // u(tau) = tau^l phi_l(tau A) v into A
            lx::LinComb lc{};
            lc.n_terms = 1;
            lc.x[0] = P[l - 1];
            lc.a[0] = std::pow(tau, l);
            LX_HIP(ctx, lx::launch_lincomb(A, nullptr, 0.0, lc, N, ctx->stream));
            const double fin = q.sigma[k] / std::pow(H, l);
            for (int j = 1; j < s; ++j) {
                const double t = j * tau;
                st = call(single(A, B, 0, tau, 1.0));   // B = e^{tau A} u(t)
                if (st != LX_OK) return st;
                iters[k] += ctx->stats.iters[0];
                errs[k] = ctx->stats.err[0];
                const bool last = j == s - 1;
                const double sc = last ? fin : 1.0;
                lx::LinComb u{};
                u.n_terms = l;
                double fact = 1.0;   // (l - i)!, from i = l down
                for (int i = l; i >= 1; --i) {
                    if (i < l) fact *= static_cast<double>(l - i);
                    u.x[i - 1] = P[i - 1];
                    u.a[i - 1] = sc * std::pow(tau, i) * std::pow(t, l - i) / fact;
                }
                double* dst = last ? q.out[k] : A;
                LX_HIP(ctx, lx::launch_lincomb(dst, B, sc, u, N, ctx->stream));
            }
        }
    }
    LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < q.K; ++k) {
        acc.iters[k] = iters[k];
        acc.err[k] = errs[k];
        const lx_status st = rms_norm(ctx, q.out[k], N, &acc.pnorm[k]);
        if (st != LX_OK) return st;
    }
    acc.substeps = s;
    acc.status = worst;
    ctx->stats = acc;
    if (worst == LX_ENOTCONV) ctx->err = "not converged within max_iters (a substep call)";
    return worst;
}

// Power iteration by register marching (power_stream): up to
// kPowerStreamDepth sweeps per launch, normalised at launch boundaries.  The
// unnormalised levels grow at most like the Gershgorin bound g of A (the
// start of a launch has norm 1), so a launch makes at most 140 / log10(g)
// levels: their squares stay below 1e280 (below 1e300 for a first launch
// that takes x0 unscaled with ||x0||^2 <= 1e20).
lx_status spectrum_stream(lx_ctx* ctx, const lx_operator& op, const double* x0, int iters, double safety,
                          double* rho_hat, double* c, double* gamma) {
    constexpr int DP = lx::kPowerStreamDepth;
    const int nx = op.nx, ny = op.ny;
    const long N = static_cast<long>(nx) * ny;
    double pk[9];
    diffadv_stencil9(op, 0.0, 1.0, pk);
    const double g = std::fabs(pk[0]) + std::fabs(pk[1]) + std::fabs(pk[2]) + std::fabs(pk[3]) + std::fabs(pk[4]);
    const int cap = g > 10.0 ? static_cast<int>(140.0 / std::log10(g)) : DP;
    const int per = std::max(1, std::min(DP, cap));
    const StreamGrid sg = stream_grid(lx::kOpDiffAdv, false, nx, ny, 1, DP, 0, 0, true);
    PowerArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.tiles_x = sg.strips;
    a.tiles_y = sg.bands;
    a.nb = sg.nb;
    a.cE = pk[0];
    a.cW = pk[1];
    a.cN = pk[2];
    a.cS = pk[3];
    a.cC = pk[4];
    lx_status s = ensure_partials(ctx, 2 * static_cast<size_t>(a.nb) * (1 + DP));
    if (s != LX_OK) return s;
    a.partials = ctx->partials;
    a.ctl = ctx->ctl;
    const int nblk = (iters + per - 1) / per;
    if (ctx->timing) {
        s = ensure_timing_events(ctx, static_cast<size_t>(nblk) + 1);
        if (s != LX_OK) return s;
    }
    // raw: the first launch takes x0 unscaled and measures its norm itself
    // (when it makes a full DP levels); a NaN estimate from it means that
    // ||x0|| lay outside the range where that is safe, and the iteration
    // runs again with x0 scaled first
    auto run = [&](const bool raw) -> lx_status {
        if (!raw) LX_HIP(ctx, lx::launch_power_norm(x0, N, a.nb, ctx->partials, ctx->stream));
        if (ctx->timing) LX_HIP(ctx, hipEventRecord(ctx->tev[0], ctx->stream));
        int nlev = per, prev = per;
        for (int b = 0; b < nblk; ++b) {
            nlev = (b == nblk - 1) ? iters - per * (nblk - 1) : per;
            const double* in = (b == 0) ? x0 : ctx->ybuf[(b - 1) & 1];
            LX_HIP(ctx, lx::launch_power_stream(a, in, ctx->ybuf[b & 1], b, nlev, prev, raw, ctx->stream));
            if (ctx->timing) LX_HIP(ctx, hipEventRecord(ctx->tev[b + 1], ctx->stream));
            prev = nlev;
        }
        LX_HIP(ctx, lx::launch_power_stream_final(a, nblk - 1, nlev, raw, ctx->stream));
        LX_HIP(ctx, hipMemcpyAsync(ctx->h_ctl, ctx->ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, ctx->stream));
        LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return LX_OK;
    };
    const bool raw = per == DP && iters >= DP;
    s = run(raw);
    if (s != LX_OK) return s;
    if (raw && !std::isfinite(ctx->h_ctl->rho)) {
        s = run(false);
        if (s != LX_OK) return s;
    }
    const double rho = ctx->h_ctl->rho;
    lx_stats& S = ctx->stats;
    S.n_apply = iters;
    S.n_launch = nblk;
    S.depth = per;
    S.marching = 1;
    S.rho_hat = rho;
    S.bytes = 16.0 * static_cast<double>(N) * nblk;
    if (ctx->timing) {
        S.loop_ms = elapsed(ctx->tev[0], ctx->tev[nblk]);
        S.sweep_ms = S.loop_ms;
        S.first_sweep_ms = elapsed(ctx->tev[0], ctx->tev[1]);
    }
    if (!std::isfinite(rho) || !(rho > 0.0))
        return fail(ctx, LX_ENONFINITE, "power iteration produced a zero or non-finite norm");
    const double lam = -safety * rho;
    if (rho_hat) *rho_hat = rho;
    if (c) *c = lam / 2.0;
    if (gamma) *gamma = -lam / 4.0;
    S.status = LX_OK;
    return LX_OK;
}

}  // namespace

lx_status lx_internal_fail(lx_ctx* ctx, lx_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return fail(ctx, s, "%s", buf);
}
lx_status lx_internal_check_op(lx_ctx* ctx, const lx_operator* op, size_t n_limit) {
    const size_t keep = ctx->n_max;
    ctx->n_max = n_limit;
    const lx_status s = check_op(ctx, op);
    ctx->n_max = keep;
    return s;
}
lx_status lx_internal_ensure_xi(lx_ctx* ctx, int M) { return ensure_xi(ctx, M); }
lx_status lx_internal_ensure_timing_events(lx_ctx* ctx, size_t n) { return ensure_timing_events(ctx, n); }
double lx_internal_elapsed(hipEvent_t a, hipEvent_t b) { return elapsed(a, b); }

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* lx_status_string(int status) {
    switch (status) {
        case LX_OK: return "LX_OK";
        case LX_EINVAL: return "LX_EINVAL";
        case LX_ENOMEM: return "LX_ENOMEM";
        case LX_ENOTCONV: return "LX_ENOTCONV";
        case LX_ENONFINITE: return "LX_ENONFINITE";
        case LX_EDEVICE: return "LX_EDEVICE";
        default: return "unknown status";
    }
}

const char* lx_last_error(const lx_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

lx_status lx_get_stats(const lx_ctx* ctx, lx_stats* out) {
    if (ctx == nullptr || out == nullptr) return LX_EINVAL;
    *out = ctx->stats;
    return LX_OK;
}

void lx_destroy(lx_ctx* ctx) {
    if (ctx == nullptr) return;
    while (!ctx->predictors.empty()) lx_predictor_destroy(ctx->predictors.back());
    (void)hipStreamSynchronize(ctx->stream);
    for (double* p : ctx->ybuf) (void)hipFree(p);
    for (double* p : ctx->ws) (void)hipFree(p);
    for (double* p : ctx->sub_ws) (void)hipFree(p);
    for (double* p : ctx->blk_ws) (void)hipFree(p);
    (void)hipFree(ctx->u32);
    (void)hipFree(ctx->partials);
    (void)hipFree(ctx->ctl);
    (void)hipFree(ctx->coef);
    (void)hipFree(ctx->xi);
    (void)hipHostFree(ctx->h_ctl);
    (void)hipHostFree(ctx->h_poll);
    (void)hipHostFree(ctx->h_coef);
    (void)hipHostFree(ctx->h_xi);
    for (hipEvent_t e : ctx->poll_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
    lx_internal_free_batch(ctx);
    delete ctx;
}

lx_status lx_create(lx_ctx** out, size_t n_max, int k_max, void* stream) {
    if (out == nullptr) return LX_EINVAL;
    *out = nullptr;
    if (n_max < 9 || k_max < 1 || k_max > LX_K_MAX) return LX_EINVAL;
    lx_ctx* ctx = new lx_ctx();
    ctx->n_max = n_max;
    ctx->k_max = k_max;
    ctx->stream = static_cast<hipStream_t>(stream);
    auto bail = [&](lx_status s) {
        lx_destroy(ctx);
        return s;
    };
    if (hipGetDevice(&ctx->device) != hipSuccess) return bail(LX_EDEVICE);
    for (auto& p : ctx->ybuf)
        if (hipMalloc(&p, sizeof(double) * n_max) != hipSuccess) return bail(LX_ENOMEM);
    if (hipMalloc(&ctx->u32, sizeof(float) * n_max) != hipSuccess) return bail(LX_ENOMEM);
    // two parity slots of (1 + k_max) partial sums per workgroup, for up to
    // 4096 workgroups (grown on demand for larger grids)
    ctx->partials_len = 2 * static_cast<size_t>(1 + k_max) * 4096;
    if (hipMalloc(&ctx->partials, sizeof(double) * ctx->partials_len) != hipSuccess) return bail(LX_ENOMEM);
    if (hipMalloc(&ctx->ctl, sizeof(LoopCtl)) != hipSuccess) return bail(LX_ENOMEM);
    if (hipMalloc(&ctx->coef, sizeof(double) * k_max * lx::kMaxPoints) != hipSuccess) return bail(LX_ENOMEM);
    if (hipMalloc(&ctx->xi, sizeof(double) * lx::kMaxPoints) != hipSuccess) return bail(LX_ENOMEM);
    if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_ctl), sizeof(LoopCtl), hipHostMallocDefault) != hipSuccess)
        return bail(LX_ENOMEM);
    if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_poll), 2 * sizeof(SweepState), hipHostMallocDefault) !=
        hipSuccess)
        return bail(LX_ENOMEM);
    if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_coef), sizeof(double) * k_max * lx::kMaxPoints,
                      hipHostMallocDefault) != hipSuccess)
        return bail(LX_ENOMEM);
    if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_xi), sizeof(double) * lx::kMaxPoints, hipHostMallocDefault) !=
        hipSuccess)
        return bail(LX_ENOMEM);
    for (auto& e : ctx->poll_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return bail(LX_EDEVICE);
    std::memset(ctx->h_ctl, 0, sizeof(LoopCtl));
    std::memset(ctx->h_poll, 0, 2 * sizeof(SweepState));
    if (hipMemcpyAsync(ctx->ctl, ctx->h_ctl, sizeof(LoopCtl), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        return bail(LX_EDEVICE);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(LX_EDEVICE);
    load_tune_cache(ctx);
    *out = ctx;
    return LX_OK;
}

lx_status lx_set_stream(lx_ctx* ctx, void* stream) {
    if (ctx == nullptr) return LX_EINVAL;
    // launches a Leja loop left queued read the loop state, which the next
    // call resets: they finish before work goes to another stream
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, LX_EDEVICE, "stream synchronisation failed");
    ctx->stream = static_cast<hipStream_t>(stream);
    return LX_OK;
}

lx_status lx_set_timing(lx_ctx* ctx, int on) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->timing = on ? 1 : 0;
    return LX_OK;
}

lx_status lx_spectrum(lx_ctx* ctx, const lx_operator* op, const double* d_u, const double* d_x0, int iters,
                      double safety, double* rho_hat, double* c, double* gamma) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = check_op(ctx, op);
    if (s != LX_OK) return s;
    if (iters < 1 || iters > LX_MAX_ITERS) return fail(ctx, LX_EINVAL, "power iterations %d outside 1..%d", iters, LX_MAX_ITERS);
    if (!(safety > 0.0) || !std::isfinite(safety)) return fail(ctx, LX_EINVAL, "safety must be finite and > 0");
    if (op->kind == LX_OP_BURGERS2D && d_u == nullptr) return fail(ctx, LX_EINVAL, "Burgers Jacobian needs d_u");
    const int nx = op->nx, ny = op->ny;
    const long N = static_cast<long>(nx) * ny;

    const double* x0 = d_x0;
    if (x0 == nullptr) {
        LX_HIP(ctx, lx::launch_fill_splitmix(ctx->ybuf[1], N, 0ull, ctx->stream));
        x0 = ctx->ybuf[1];
    }
    const bool vec2 = aligned16(x0) && (d_u == nullptr || aligned16(d_u));
    // kPowerBlockDepth sweeps per launch on LDS tiles (the basis read and
    // written once per launch, the Burgers state once per launch); odd or
    // narrow grids and unaligned vectors one sweep per launch
    if (ctx->win_kind != 1 && op->kind == LX_OP_DIFFADV2D && vec2 && nx % 2 == 0 && nx >= lx::kPowerStreamDepth &&
        ny >= lx::kPowerStreamDepth && N * 8 <= (1L << 30))
        return spectrum_stream(ctx, *op, x0, iters, safety, rho_hat, c, gamma);
    constexpr int PD = lx::kPowerBlockDepth;
    const int pcode = opcode_of(op->kind);
    const int ph = PD * (op->kind == LX_OP_DIFFADV2D_UP3 ? 2 : 1);   // halo of a power launch
    if (vec2 && nx % 2 == 0 && nx >= ph && ny >= ph) {
        const int prow = lx::power_block_rows(pcode);
        PowerArgs a{};
        a.nx = nx;
        a.ny = ny;
        a.tiles_x = (nx + 127) / 128;
        a.tiles_y = (ny + prow - 1) / prow;
        // one resident round of workgroups: a grid larger than what fits at
        // once leaves a partial second round (1024 workgroups of 52 KB of LDS
        // on 256 CUs that hold three each)
        const int resident = lx::power_block_resident(pcode);
        a.nb = pair_grid(resident > 0 ? resident : 1024, a.tiles_x * a.tiles_y);
        if (is_diffadv(op->kind)) {
            double pk[9];
            diffadv_stencil9(*op, 0.0, 1.0, pk);
            a.cE = pk[0];
            a.cW = pk[1];
            a.cN = pk[2];
            a.cS = pk[3];
            a.cC = pk[4];
            a.cE2 = pk[5];
            a.cW2 = pk[6];
            a.cN2 = pk[7];
            a.cS2 = pk[8];
        } else {
            double pk[5];
            lx::stencil_coeffs(1, op->dx, op->dy, op->D, op->vx, op->vy, op->nu, 0.0, 1.0, pk);
            a.kx = pk[0];
            a.ky = pk[1];
            a.gx = pk[2];
            a.gy = pk[3];
            a.u = d_u;
        }
        s = ensure_partials(ctx, 2 * static_cast<size_t>(a.nb) * (1 + PD));
        if (s != LX_OK) return s;
        a.partials = ctx->partials;
        a.ctl = ctx->ctl;
        const int nblk = (iters + PD - 1) / PD;
        LX_HIP(ctx, lx::launch_power_norm(x0, N, a.nb, ctx->partials, ctx->stream));
        if (ctx->timing) {
            s = ensure_timing_events(ctx, static_cast<size_t>(nblk) + 1);
            if (s != LX_OK) return s;
            LX_HIP(ctx, hipEventRecord(ctx->tev[0], ctx->stream));
        }
        int nlev = PD;
        for (int b = 0; b < nblk; ++b) {
            nlev = (b == nblk - 1) ? iters - PD * (nblk - 1) : PD;
            const double* in = (b == 0) ? x0 : ctx->ybuf[(b - 1) & 1];
            LX_HIP(ctx, lx::launch_power_block(pcode, a, in, ctx->ybuf[b & 1], b, nlev, ctx->stream));
            if (ctx->timing) LX_HIP(ctx, hipEventRecord(ctx->tev[b + 1], ctx->stream));
        }
        LX_HIP(ctx, lx::launch_power_block_final(a, nblk - 1, nlev, ctx->stream));
        LX_HIP(ctx, hipMemcpyAsync(ctx->h_ctl, ctx->ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, ctx->stream));
        LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const double rho = ctx->h_ctl->rho;
        lx_stats& S = ctx->stats;
        S.n_apply = iters;
        S.n_launch = nblk;
        S.depth = PD;
        S.rho_hat = rho;
        S.bytes = (op->kind == LX_OP_BURGERS2D ? 24.0 : 16.0) * static_cast<double>(N) * nblk;   // + u per launch
        if (ctx->timing) {
            S.loop_ms = elapsed(ctx->tev[0], ctx->tev[nblk]);
            S.sweep_ms = S.loop_ms;
            S.first_sweep_ms = elapsed(ctx->tev[0], ctx->tev[1]);
        }
        if (!std::isfinite(rho) || !(rho > 0.0))
            return fail(ctx, LX_ENONFINITE, "power iteration produced a zero or non-finite norm");
        const double lam = -safety * rho;
        if (rho_hat) *rho_hat = rho;
        if (c) *c = lam / 2.0;
        if (gamma) *gamma = -lam / 4.0;
        S.status = LX_OK;
        return LX_OK;
    }
    const Tile t = pick_tile(ctx, *op, 1, vec2);
    PowerArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.tiles_x = (nx + t.cols() - 1) / t.cols();
    a.tiles_y = (ny + t.rows() - 1) / t.rows();
    a.nb = grid_size(t, a.tiles_x * a.tiles_y);
    if (is_diffadv(op->kind)) {
        double pk[9];
        diffadv_stencil9(*op, 0.0, 1.0, pk);
        a.cE = pk[0];
        a.cW = pk[1];
        a.cN = pk[2];
        a.cS = pk[3];
        a.cC = pk[4];
        a.cE2 = pk[5];
        a.cW2 = pk[6];
        a.cN2 = pk[7];
        a.cS2 = pk[8];
    } else {
        double pk[5];
        lx::stencil_coeffs(1, op->dx, op->dy, op->D, op->vx, op->vy, op->nu, 0.0, 1.0, pk);
        a.kx = pk[0];
        a.ky = pk[1];
        a.gx = pk[2];
        a.gy = pk[3];
    }
    a.u = d_u;
    s = ensure_partials(ctx, 2 * static_cast<size_t>(a.nb));
    if (s != LX_OK) return s;
    a.partials = ctx->partials;
    a.ctl = ctx->ctl;
    const int opcode = opcode_of(op->kind);
    // |x0|^2 partials into slot 1, read by sweep 0
    LX_HIP(ctx, lx::launch_power_norm(x0, N, a.nb, ctx->partials, ctx->stream));
    if (ctx->timing) {
        s = ensure_timing_events(ctx, static_cast<size_t>(iters) + 1);
        if (s != LX_OK) return s;
        LX_HIP(ctx, hipEventRecord(ctx->tev[0], ctx->stream));
    }
    for (int k = 0; k < iters; ++k) {
        a.in = (k == 0) ? x0 : ctx->ybuf[(k - 1) & 1];
        a.out = ctx->ybuf[k & 1];
        LX_HIP(ctx, lx::launch_power_sweep(opcode, t, a, k, ctx->stream));
        if (ctx->timing) LX_HIP(ctx, hipEventRecord(ctx->tev[k + 1], ctx->stream));
    }
    LX_HIP(ctx, lx::launch_power_final(a.nb, ctx->partials + static_cast<size_t>((iters - 1) & 1) * a.nb, ctx->ctl,
                                       ctx->stream));
    LX_HIP(ctx, hipMemcpyAsync(ctx->h_ctl, ctx->ctl, sizeof(LoopCtl), hipMemcpyDeviceToHost, ctx->stream));
    LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double rho = ctx->h_ctl->rho;
    lx_stats& S = ctx->stats;
    S.n_apply = iters;
    S.n_launch = iters;
    S.depth = 1;
    S.rho_hat = rho;
    S.bytes = (16.0 + (op->kind == LX_OP_BURGERS2D ? 8.0 : 0.0)) * static_cast<double>(N) * iters;
    if (ctx->timing) {
        S.loop_ms = elapsed(ctx->tev[0], ctx->tev[iters]);
        S.sweep_ms = S.loop_ms;
        S.first_sweep_ms = elapsed(ctx->tev[0], ctx->tev[1]);
    }
    if (!std::isfinite(rho) || !(rho > 0.0))
        return fail(ctx, LX_ENONFINITE, "power iteration produced a zero or non-finite norm");
    const double lam = -safety * rho;
    if (rho_hat) *rho_hat = rho;
    if (c) *c = lam / 2.0;
    if (gamma) *gamma = -lam / 4.0;
    S.status = LX_OK;
    return LX_OK;
}

lx_status lx_phi_leja(lx_ctx* ctx, const lx_operator* op, const double* d_u, const double* d_v, int K, const int* l,
                      const double* alpha, const double* sigma, double* const* d_out, double h, double c,
                      double gamma, const lx_leja_opts* o, int* iters, double* err) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = check_op(ctx, op);
    if (s != LX_OK) return s;
    if (K < 1 || K > ctx->k_max) return fail(ctx, LX_EINVAL, "K = %d outside 1..%d", K, ctx->k_max);
    if (d_v == nullptr || d_out == nullptr || l == nullptr) return fail(ctx, LX_EINVAL, "NULL vector or order array");
    if (op->kind == LX_OP_BURGERS2D && d_u == nullptr) return fail(ctx, LX_EINVAL, "Burgers Jacobian needs d_u");
    s = check_shift(ctx, h, c, gamma);
    if (s != LX_OK) return s;
    LejaCall q{};
    s = check_leja_opts(ctx, o, &q.o);
    if (s != LX_OK) return s;
    q.op = op;
    q.u = op->kind == LX_OP_BURGERS2D ? d_u : nullptr;
    q.v = d_v;
    q.K = K;
    q.h = h;
    q.c = c;
    q.gamma = gamma;
    for (int k = 0; k < K; ++k) {
        if (l[k] < 0 || l[k] > 8) return fail(ctx, LX_EINVAL, "phi order l[%d] = %d outside 0..8", k, l[k]);
        q.l[k] = l[k];
        q.alpha[k] = alpha ? alpha[k] : 1.0;
        q.sigma[k] = sigma ? sigma[k] : 1.0;
        if (!(q.alpha[k] > 0.0) || !std::isfinite(q.alpha[k]) || !std::isfinite(q.sigma[k]))
            return fail(ctx, LX_EINVAL, "alpha[%d] must be finite and > 0, sigma finite", k);
        if (d_out[k] == nullptr) return fail(ctx, LX_EINVAL, "d_out[%d] is NULL", k);
        if (d_out[k] == d_v || (q.u != nullptr && d_out[k] == q.u))
            return fail(ctx, LX_EINVAL, "d_out[%d] aliases an input", k);
        for (int j = 0; j < k; ++j)
            if (d_out[j] == d_out[k]) return fail(ctx, LX_EINVAL, "d_out[%d] and d_out[%d] alias", j, k);
        q.out[k] = d_out[k];
    }
    s = run_leja_sub(ctx, q);
    for (int k = 0; k < K; ++k) {
        if (iters) iters[k] = ctx->stats.iters[k];
        if (err) err[k] = ctx->stats.err[k];
    }
    return s;
}

lx_status lx_phi_leja_static(lx_ctx* ctx, const lx_operator* op, const double* d_u, const double* d_v, int K,
                             const int* l, const double* alpha, const double* sigma, double* const* d_out, double h,
                             double c, double gamma, const lx_leja_opts* o, int* iters, double* err) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = lx_internal_check_op(ctx, op, lx::kStaticPoints);
    if (s != LX_OK) return s;
    if (op->prec != LX_FP64) return fail(ctx, LX_EINVAL, "lx_phi_leja_static runs FP64 sweeps only");
    if (K < 1 || K > ctx->k_max) return fail(ctx, LX_EINVAL, "K = %d outside 1..%d", K, ctx->k_max);
    if (d_v == nullptr || d_out == nullptr || l == nullptr) return fail(ctx, LX_EINVAL, "NULL vector or order array");
    if (op->kind == LX_OP_BURGERS2D && d_u == nullptr) return fail(ctx, LX_EINVAL, "Burgers Jacobian needs d_u");
    s = check_shift(ctx, h, c, gamma);
    if (s != LX_OK) return s;
    LejaCall q{};
    s = check_leja_opts(ctx, o, &q.o);
    if (s != LX_OK) return s;
    q.op = op;
    q.u = op->kind == LX_OP_BURGERS2D ? d_u : nullptr;
    q.v = d_v;
    q.K = K;
    q.h = h;
    q.c = c;
    q.gamma = gamma;
    double amax = 0.0;
    for (int k = 0; k < K; ++k) {
        if (l[k] < 0 || l[k] > 8) return fail(ctx, LX_EINVAL, "phi order l[%d] = %d outside 0..8", k, l[k]);
        q.l[k] = l[k];
        q.alpha[k] = alpha ? alpha[k] : 1.0;
        q.sigma[k] = sigma ? sigma[k] : 1.0;
        if (!(q.alpha[k] > 0.0) || !std::isfinite(q.alpha[k]) || !std::isfinite(q.sigma[k]))
            return fail(ctx, LX_EINVAL, "alpha[%d] must be finite and > 0, sigma finite", k);
        if (d_out[k] == nullptr) return fail(ctx, LX_EINVAL, "d_out[%d] is NULL", k);
        if (d_out[k] == d_v || (q.u != nullptr && d_out[k] == q.u))
            return fail(ctx, LX_EINVAL, "d_out[%d] aliases an input", k);
        for (int j = 0; j < k; ++j)
            if (d_out[j] == d_out[k]) return fail(ctx, LX_EINVAL, "d_out[%d] and d_out[%d] alias", j, k);
        q.out[k] = d_out[k];
        amax = std::max(amax, q.alpha[k]);
    }
    // one Leja call: substeps would need more workspace vectors
    const int sub = q.o.substeps != 0 ? q.o.substeps
                                      : static_cast<int>(std::max(1.0, std::ceil(amax * h * gamma / kSubstepHGamma)));
    if (sub != 1) return fail(ctx, LX_EINVAL, "lx_phi_leja_static takes no substeps (this call would need %d)", sub);
    // the library's static device scratch on the current device
    int dev = 0;
    LX_HIP(ctx, hipGetDevice(&dev));
    LX_HIP(ctx, lx::static_scratch(dev, &q.scratch));
    s = run_leja(ctx, q);
    for (int k = 0; k < K; ++k) {
        if (iters) iters[k] = ctx->stats.iters[k];
        if (err) err[k] = ctx->stats.err[k];
    }
    return s;
}

lx_status lx_linear_step(lx_ctx* ctx, const lx_operator* op, const double* d_u, const double* d_src,
                         double* d_u_out, double h, double c, double gamma, const lx_leja_opts* o, int* iters) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = check_op(ctx, op);
    if (s != LX_OK) return s;
    if (!is_diffadv(op->kind)) return fail(ctx, LX_EINVAL, "linear steps need a diffusion-advection operator");
    if (d_u == nullptr || d_u_out == nullptr || d_u == d_u_out || d_src == d_u_out)
        return fail(ctx, LX_EINVAL, "d_u and d_u_out must be distinct, non-NULL, and d_u_out must differ from d_src");
    s = check_shift(ctx, h, c, gamma);
    if (s != LX_OK) return s;
    lx_leja_opts oo;
    s = check_leja_opts(ctx, o, &oo);
    if (s != LX_OK) return s;
    const int nx = op->nx, ny = op->ny;
    const long N = static_cast<long>(nx) * ny;
    LejaCall q{};
    q.op = op;
    q.u = nullptr;
    q.K = 1;
    q.alpha[0] = 1.0;
    q.sigma[0] = 1.0;
    q.out[0] = d_u_out;
    q.h = h;
    q.c = c;
    q.gamma = gamma;
    q.o = oo;
    if (d_src == nullptr) {
        // Problem I: the exp action of u
        q.l[0] = 0;
        q.v = d_u;
        s = run_leja_sub(ctx, q);
    } else {
        // Problem II: u + phi_1(h A) h (A u + S)
        if (ctx->ws[0] == nullptr && hipMalloc(&ctx->ws[0], sizeof(double) * ctx->n_max) != hipSuccess)
            return fail(ctx, LX_ENOMEM, "linear-step workspace allocation failed");
        // h (A u + S) with the power sweep's tiles and shape
        double k9[9];
        diffadv_stencil9(*op, 0.0, 1.0, k9);
        const bool vec2 = aligned16(d_u) && aligned16(d_src) && aligned16(ctx->ws[0]);
        const Tile t = pick_tile(ctx, *op, 1, vec2);
        PowerArgs a{};
        a.nx = nx;
        a.ny = ny;
        a.tiles_x = (nx + t.cols() - 1) / t.cols();
        a.tiles_y = (ny + t.rows() - 1) / t.rows();
        a.nb = grid_size(t, a.tiles_x * a.tiles_y);
        a.cE = k9[0];
        a.cW = k9[1];
        a.cN = k9[2];
        a.cS = k9[3];
        a.cC = k9[4];
        a.cE2 = k9[5];
        a.cW2 = k9[6];
        a.cN2 = k9[7];
        a.cS2 = k9[8];
        a.in = d_u;
        a.out = ctx->ws[0];
        a.add = d_src;
        LX_HIP(ctx, lx::launch_rhs_sweep(opcode_of(op->kind), t, a, h, ctx->stream));
        q.l[0] = 1;
        q.v = ctx->ws[0];
        s = run_leja_sub(ctx, q);
        if (s == LX_OK || s == LX_ENOTCONV) {
            // after LX_ENOTCONV too: u plus the last polynomial
            LX_HIP(ctx, lx::launch_combine(d_u, d_u_out, nullptr, d_u_out, N, ctx->stream));
            LX_HIP(ctx, hipStreamSynchronize(ctx->stream));
        }
    }
    if (iters) *iters = ctx->stats.iters[0];
    return s;
}

lx_status lx_exprb_step(lx_ctx* ctx, const lx_operator* op, int scheme, const double* d_u, double* d_u_out,
                        double* d_u_low, double* err, double h, double c, double gamma, const lx_leja_opts* o,
                        int* iters) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = check_op(ctx, op);
    if (s != LX_OK) return s;
    if (op->kind != LX_OP_BURGERS2D) return fail(ctx, LX_EINVAL, "exponential integrator steps need LX_OP_BURGERS2D");
    if (scheme != LX_ROS_EULER && scheme != LX_EXPRB32 && scheme != LX_EXPRB42)
        return fail(ctx, LX_EINVAL, "unknown scheme %d", scheme);
    if (d_u == nullptr || d_u_out == nullptr || d_u == d_u_out)
        return fail(ctx, LX_EINVAL, "d_u and d_u_out must be distinct, non-NULL");
    if (d_u_low != nullptr && scheme != LX_EXPRB32)
        return fail(ctx, LX_EINVAL, "d_u_low: only LX_EXPRB32 has an embedded lower-order solution");
    if (d_u_low != nullptr && (d_u_low == d_u || d_u_low == d_u_out))
        return fail(ctx, LX_EINVAL, "d_u_low must differ from d_u and d_u_out");
    if (scheme == LX_EXPRB42 && ctx->k_max < 2) return fail(ctx, LX_EINVAL, "EXPRB42 needs a context with k_max >= 2");
    s = check_shift(ctx, h, c, gamma);
    if (s != LX_OK) return s;
    lx_leja_opts oo;
    s = check_leja_opts(ctx, o, &oo);
    if (s != LX_OK) return s;
    for (auto& w : ctx->ws)
        if (w == nullptr && hipMalloc(&w, sizeof(double) * ctx->n_max) != hipSuccess)
            return fail(ctx, LX_ENOMEM, "integrator workspace allocation failed");
    const int nx = op->nx, ny = op->ny;
    const long N = static_cast<long>(nx) * ny;
    double* hF = ctx->ws[0];   // h F(u), later the remainder h [N(u + a) - N(u)]
    auto pass = [&](int K, const int* l, const double* alpha, const double* sigma, double* const* out,
                    const double* v) -> lx_status {
        LejaCall q{};
        q.op = op;
        q.u = d_u;
        q.v = v;
        q.K = K;
        for (int k = 0; k < K; ++k) {
            q.l[k] = l[k];
            q.alpha[k] = alpha[k];
            q.sigma[k] = sigma[k];
            q.out[k] = out[k];
        }
        q.h = h;
        q.c = c;
        q.gamma = gamma;
        q.o = oo;
        return run_leja_sub(ctx, q);
    };
    auto merge = [](lx_stats& acc, const lx_stats& t) {
        acc.n_apply += t.n_apply;
        acc.n_fp32 += t.n_fp32;
        acc.n_launch += t.n_launch;
        acc.plan_ms += t.plan_ms;
        acc.loop_ms += t.loop_ms;
        acc.sweep_ms += t.sweep_ms;
        acc.bytes += t.bytes;
        acc.depth = t.depth;
        acc.marching = t.marching;
    };
    LX_HIP(ctx, lx::launch_burgers_hF(d_u, hF, nx, ny, op->nu, op->dx, op->dy, h, ctx->stream));
    lx_stats acc{};
    int it[3] = {0, 0, 0};   // every phi action of the step, in the order taken
    double e1 = 0.0, e2 = 0.0, step_err = 0.0;
    if (scheme == LX_ROS_EULER) {
        // u+ = u + phi_1(h J) h F(u)
        const int l[1] = {1};
        const double one[1] = {1.0};
        double* out[1] = {d_u_out};
        s = pass(1, l, one, one, out, hF);
        if (s != LX_OK) return s;
        acc = ctx->stats;
        it[0] = acc.iters[0];
        e1 = acc.err[0];
        LX_HIP(ctx, lx::launch_combine(d_u, d_u_out, nullptr, d_u_out, N, ctx->stream));
    } else if (scheme == LX_EXPRB32) {
        // a = u + phi_1(h J) h F(u);  u+ = a + 2 phi_3(h J) h [N(a) - N(u)];
        // the embedded estimate is the rms norm of the correction
        // (the embedded second-order solution a goes to d_u_low when given)
        double* p1 = ctx->ws[1];
        double* a = d_u_low != nullptr ? d_u_low : ctx->ws[2];
        const int l1[1] = {1}, l3[1] = {3};
        const double one[1] = {1.0}, two[1] = {2.0};
        double* out1[1] = {p1};
        s = pass(1, l1, one, one, out1, hF);
        if (s != LX_OK) return s;
        acc = ctx->stats;
        it[0] = acc.iters[0];
        e1 = acc.err[0];
        LX_HIP(ctx, lx::launch_combine(d_u, p1, nullptr, a, N, ctx->stream));
        LX_HIP(ctx, lx::launch_burgers_remainder(d_u, p1, hF, nx, ny, op->nu, op->dx, op->dy, h, ctx->stream));
        double* out2[1] = {d_u_out};
        s = pass(1, l3, one, two, out2, hF);
        const lx_stats t = ctx->stats;
        merge(acc, t);
        it[1] = t.iters[0];
        e2 = t.err[0];
        step_err = t.pnorm[0];
        if (s != LX_OK) {
            ctx->stats = acc;
            return s;
        }
        LX_HIP(ctx, lx::launch_combine(a, d_u_out, nullptr, d_u_out, N, ctx->stream));
    } else {
        // one Newton basis for (3/4) h phi_1((3/4) h J) F(u) and h phi_1(h J) F(u);
        // U2 = u + the first; u+ = u + the second + (32/9) h phi_3(h J) [N(U2) - N(u)]
        double* a = ctx->ws[1];
        double* p1 = ctx->ws[2];
        const int l1[2] = {1, 1}, l3[1] = {3};
        const double alpha1[2] = {0.75, 1.0}, sigma1[2] = {0.75, 1.0};
        const double one[1] = {1.0}, s3[1] = {32.0 / 9.0};
        double* out1[2] = {a, p1};
        s = pass(2, l1, alpha1, sigma1, out1, hF);
        if (s != LX_OK) return s;
        acc = ctx->stats;
        it[0] = acc.iters[0];
        it[1] = acc.iters[1];
        e1 = std::max(acc.err[0], acc.err[1]);
        LX_HIP(ctx, lx::launch_burgers_remainder(d_u, a, hF, nx, ny, op->nu, op->dx, op->dy, h, ctx->stream));
        double* out2[1] = {d_u_out};
        s = pass(1, l3, one, s3, out2, hF);
        const lx_stats t = ctx->stats;
        merge(acc, t);
        it[2] = t.iters[0];
        e2 = t.err[0];
        if (s != LX_OK) {
            ctx->stats = acc;
            return s;
        }
        LX_HIP(ctx, lx::launch_combine(d_u, p1, d_u_out, d_u_out, N, ctx->stream));
    }
    if (iters) {
        for (int i = 0; i < 3; ++i) iters[i] = it[i];
    }
    if (err) *err = step_err;
    for (int i = 0; i < 3; ++i) acc.iters[i] = it[i];
    acc.iters[3] = 0;
    acc.err[0] = e1;
    acc.err[1] = e2;
    acc.step_err = step_err;
    acc.status = LX_OK;
    ctx->stats = acc;
    return LX_OK;
}

lx_status lx_set_depth(lx_ctx* ctx, int depth, int th, int nb) {
    if (ctx == nullptr) return LX_EINVAL;
    if (depth < 0 || depth == 5 || depth == 7 || depth > 8 || !(th == 0 || th == 8 || th == 16 || th == 32) || nb < 0)
        return fail(ctx, LX_EINVAL, "depth %d, th %d, nb %d: need depth 0..4, 6 or 8, th 0/8/16/32, nb >= 0", depth,
                    th, nb);
    ctx->depth_forced = depth;
    ctx->pair_th = th;
    ctx->pair_nb = nb;
    return LX_OK;
}

lx_status lx_set_window_kernel(lx_ctx* ctx, int kind, int bands, int nb) {
    if (ctx == nullptr) return LX_EINVAL;
    if (kind < 0 || kind > 2 || bands < 0 || nb < 0)
        return fail(ctx, LX_EINVAL, "window kernel %d, bands %d, nb %d: need kind 0..2, bands >= 0, nb >= 0", kind,
                    bands, nb);
    ctx->win_kind = kind;
    ctx->win_bands = bands;
    ctx->win_nb = nb;
    return LX_OK;
}

lx_status lx_set_tile(lx_ctx* ctx, int tx, int ty, int ry, int vec, int nb) {
    if (ctx == nullptr) return LX_EINVAL;
    if (tx == 0) {
        ctx->forced = Tile{0, 0, 0, 0, 0};
        return LX_OK;
    }
    const Tile t{tx, ty, ry, vec, nb};
    if (!valid_tile(t))
        return fail(ctx, LX_EINVAL, "invalid launch shape tx=%d ty=%d ry=%d vec=%d nb=%d", tx, ty, ry, vec, nb);
    ctx->forced = t;
    return LX_OK;
}

lx_status lx_tune(lx_ctx* ctx, const lx_operator* op, int K, int sweeps, char* report, size_t report_len) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    lx_status s = check_op(ctx, op);
    if (s != LX_OK) return s;
    if (K < 1 || K > ctx->k_max) return fail(ctx, LX_EINVAL, "K = %d outside 1..%d", K, ctx->k_max);
    if (sweeps < 1 || sweeps > 200) return fail(ctx, LX_EINVAL, "sweeps %d outside 1..200", sweeps);
    const int nx = op->nx, ny = op->ny;
    const size_t N = static_cast<size_t>(nx) * ny;
    const int ld = sweeps + 16;   // windows read up to 2 depths past the timed sweeps
    s = ensure_xi(ctx, ld);
    if (s != LX_OK) return s;
    // scratch: K outputs (+ the Burgers state), all zero, so that values stay
    // finite for any number of sweeps; atol < 0 keeps the loop running
    double* scratch = nullptr;
    const size_t nvec = static_cast<size_t>(K) + (op->kind == LX_OP_BURGERS2D ? 1 : 0);
    if (hipMalloc(&scratch, sizeof(double) * N * nvec) != hipSuccess) return fail(ctx, LX_ENOMEM, "tuning scratch");
    auto cleanup = [&](lx_status r) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(scratch);
        return r;
    };
    if (hipMemsetAsync(scratch, 0, sizeof(double) * N * nvec, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->ybuf[0], 0, sizeof(double) * N, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->ybuf[1], 0, sizeof(double) * N, ctx->stream) != hipSuccess)
        return cleanup(fail(ctx, LX_EDEVICE, "tuning scratch clear failed"));
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < ld; ++j) ctx->h_coef[static_cast<size_t>(k) * ld + j] = 1e-3;
    if (hipMemcpyAsync(ctx->coef, ctx->h_coef, sizeof(double) * K * ld, hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
        return cleanup(fail(ctx, LX_EDEVICE, "coefficient upload failed"));
    LoopCtl& init = *ctx->h_ctl;
    std::memset(&init, 0, sizeof(init));
    init.max_iters = LX_MAX_ITERS;
    init.rtol = 0.0;
    init.atol = -1.0;
    // FP32 sweeps are timed in FP32 from the first sweep
    init.fp32_switch = op->prec == LX_FP32_SWEEP ? 0.0 : -1.0;
    init.slot[0].out32 = op->prec == LX_FP32_SWEEP ? 1 : 0;
    for (int k = 0; k < K; ++k) {
        init.slot[0].active[k] = 1;
        init.slot[0].iters[k] = LX_MAX_ITERS;
    }
    if (op->prec == LX_FP32_SWEEP && hipMemsetAsync(ctx->u32, 0, sizeof(float) * N, ctx->stream) != hipSuccess)
        return cleanup(fail(ctx, LX_EDEVICE, "tuning scratch clear failed"));
    s = ensure_timing_events(ctx, 2);
    if (s != LX_OK) return cleanup(s);

    const bool vec2_ok = nx % 2 == 0;
    std::vector<Tile> cands;
    for (int tx : {64, 32, 16, 8, 4}) {
        Tile t;
        t.tx = tx;
        t.ty = lx::kBlockThreads / tx;
        t.vec = vec2_ok ? 2 : 1;
        if (t.cols() > nx && tx > 4) continue;   // narrower workgroups cover this grid
        for (int ry : {1, 2, 4, 8}) {
            t.ry = ry;
            if (t.rows() > ny && ry > 1) continue;
            const int tiles = tiles_of(t, nx, ny);
            for (int nb : {0, 2048, 1024, 512}) {
                if (nb != 0 && nb >= tiles) continue;   // same as one workgroup per tile
                t.nb = nb;
                cands.push_back(t);
            }
        }
    }
    std::string rep;
    double best_us = 1e300;
    Tile best = cands.empty() ? choose_tile(nx, ny, vec2_ok) : cands[0];
    const int opcode = opcode_of(op->kind);
    const bool fp32 = op->prec == LX_FP32_SWEEP;
    for (const Tile& t : cands) {
        SweepArgs a{};
        a.nx = nx;
        a.ny = ny;
        a.tiles_x = (nx + t.cols() - 1) / t.cols();
        a.tiles_y = (ny + t.rows() - 1) / t.rows();
        a.nb = grid_size(t, a.tiles_x * a.tiles_y);
        a.ld = ld;
        set_stencil(a, *op, -2.0, 1.0);
        a.inv_sqrtN = 1.0 / std::sqrt(static_cast<double>(N));
        a.v = ctx->ybuf[0];
        a.ybuf[0] = ctx->ybuf[0];
        a.ybuf[1] = ctx->ybuf[1];
        a.u = op->kind == LX_OP_BURGERS2D ? scratch + static_cast<size_t>(K) * N : nullptr;
        a.u32 = ctx->u32;
        for (int k = 0; k < K; ++k) a.p[k] = scratch + static_cast<size_t>(k) * N;
        a.coef = ctx->coef;
        a.xi = ctx->xi;
        s = ensure_partials(ctx, 2 * static_cast<size_t>(a.nb) * (1 + K));
        if (s != LX_OK) return cleanup(s);
        a.partials = ctx->partials;
        a.ctl = ctx->ctl;
        if (hipMemcpyAsync(ctx->ctl, &init, sizeof(LoopCtl), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
            return cleanup(fail(ctx, LX_EDEVICE, "state upload failed"));
        // sweeps 0 and 1 warm up, sweeps 2 .. sweeps+1 are timed
        hipError_t e = hipSuccess;
        for (int m = 0; m < 2 && e == hipSuccess; ++m) e = lx::launch_leja_sweep(opcode, K, fp32, t, a, m, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(ctx->tev[0], ctx->stream);
        for (int m = 2; m < sweeps + 2 && e == hipSuccess; ++m)
            e = lx::launch_leja_sweep(opcode, K, fp32, t, a, m, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(ctx->tev[1], ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ctx->tev[1]);
        if (e != hipSuccess) return cleanup(fail(ctx, LX_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e)));
        const double us = elapsed(ctx->tev[0], ctx->tev[1]) * 1e3 / sweeps;
        char line[112];
        std::snprintf(line, sizeof(line), "1 %d %d %d %d %d %.3f\n", t.tx, t.ty, t.ry, t.vec, a.nb, us);
        rep += line;
        if (us < best_us) {
            best_us = us;
            best = t;
        }
    }
    // several iterations per launch (even nx): in FP64, two iterations and
    // LDS-tile windows, depth x tile rows x workgroups; register-marching
    // windows (FP64 or FP32 sweeps), depth x bands
    best.depth = 1;
    double best_pair_us = 1e300;
    if (nx % 2 == 0) {
        const int tiles_x = (nx + 127) / 128;
        for (int depth : {2, 3, 4, 6}) {
            if (op->prec != LX_FP64) break;
            if (depth == 6 && op->kind != LX_OP_DIFFADV2D) continue;
            const int halo = depth * (op->kind == LX_OP_DIFFADV2D_UP3 ? 2 : 1);
            if (depth >= 3 && (nx < halo || ny < halo)) continue;
            if (depth >= 3) {
                s = ensure_blk_ws(ctx, K);
                if (s != LX_OK) return cleanup(s);
            }
            for (int th : {8, 16, 32}) {
                // radius 2, and two LDS levels of windows: at most 16 rows
                if (th > 16 && (op->kind == LX_OP_DIFFADV2D_UP3 || depth >= 3)) continue;
                const int tiles = tiles_x * ((ny + th - 1) / th);
                for (int pnb : {0, 2048, 1536, 1024, 768, 512, 256}) {
                    if (pnb != 0 && pnb >= tiles) continue;
                    if (depth >= 3 && pnb > 1024) continue;
                    SweepArgs a{};
                    a.nx = nx;
                    a.ny = ny;
                    a.tiles_x = tiles_x;
                    a.tiles_y = (ny + th - 1) / th;
                    a.nb = pair_grid(pnb, tiles);
                    a.ld = ld;
                    set_stencil(a, *op, -2.0, 1.0);
                    a.inv_sqrtN = 1.0 / std::sqrt(static_cast<double>(N));
                    a.v = ctx->ybuf[0];
                    a.ybuf[0] = ctx->ybuf[0];
                    a.ybuf[1] = ctx->ybuf[1];
                    a.u = op->kind == LX_OP_BURGERS2D ? scratch + static_cast<size_t>(K) * N : nullptr;
                    for (int k = 0; k < K; ++k) a.p[k] = scratch + static_cast<size_t>(k) * N;
                    if (depth >= 3)
                        for (int k = 0; k < K; ++k) a.p2[k] = ctx->blk_ws[k];
                    a.coef = ctx->coef;
                    a.xi = ctx->xi;
                    s = ensure_partials(ctx, 2 * static_cast<size_t>(depth) * a.nb * (1 + K));
                    if (s != LX_OK) return cleanup(s);
                    a.partials = ctx->partials;
                    a.ctl = ctx->ctl;
                    if (hipMemcpyAsync(ctx->ctl, &init, sizeof(LoopCtl), hipMemcpyHostToDevice, ctx->stream) !=
                        hipSuccess)
                        return cleanup(fail(ctx, LX_EDEVICE, "state upload failed"));
                    auto go = [&](int L) {
                        return depth >= 3 ? lx::launch_leja_block(opcode, K, th, depth, a, L, ctx->stream)
                                          : lx::launch_leja_pair(opcode, K, th, a, L, ctx->stream);
                    };
                    // launches 0 and 1 warm up; launches 2 .. n+1 (depth * n iterations) are timed
                    const int n = std::max(1, sweeps / depth);
                    hipError_t e = hipSuccess;
                    for (int L = 0; L < 2 && e == hipSuccess; ++L) e = go(L);
                    if (e == hipSuccess) e = hipEventRecord(ctx->tev[0], ctx->stream);
                    for (int L = 2; L < n + 2 && e == hipSuccess; ++L) e = go(L);
                    if (e == hipSuccess) e = hipEventRecord(ctx->tev[1], ctx->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(ctx->tev[1]);
                    if (e != hipSuccess)
                        return cleanup(fail(ctx, LX_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e)));
                    const double us = elapsed(ctx->tev[0], ctx->tev[1]) * 1e3 / (static_cast<double>(depth) * n);
                    char line[112];
                    std::snprintf(line, sizeof(line), "%d 64 4 %d 2 %d %.3f\n", depth, th, a.nb, us);
                    rep += line;
                    if (us < best_pair_us) {
                        best_pair_us = us;
                        best.th = th;
                        best.pnb = pnb;
                        best.depth = depth;
                        best.stream = 0;
                    }
                }
            }
        }
        // windows by register marching (the five-point operators; FP32 sweeps
        // timed in FP32 throughout): depth x bands (one resident round, two
        // rounds, and bands of 64 and 128 rows)
        for (int depth : {4, 6, 8}) {
            if (!stream_ok(*op, K, depth)) continue;
            s = ensure_blk_ws(ctx, K);
            if (s != LX_OK) return cleanup(s);
            const StreamGrid g0 = stream_grid(opcode, fp32, nx, ny, K, depth, 0, 0, false);
            int prev_bands = -1;
            for (int bands : {g0.bands, 2 * g0.bands, ny / 64, ny / 128}) {
                if (bands < 1 || bands > ny || bands == prev_bands) continue;
                prev_bands = bands;
                const StreamGrid g = stream_grid(opcode, fp32, nx, ny, K, depth, bands, 0, false);
                SweepArgs a{};
                a.nx = nx;
                a.ny = ny;
                a.tiles_x = g.strips;
                a.tiles_y = g.bands;
                a.nb = g.nb;
                a.ld = ld;
                set_stencil(a, *op, -2.0, 1.0);
                a.inv_sqrtN = 1.0 / std::sqrt(static_cast<double>(N));
                a.v = ctx->ybuf[0];
                a.ybuf[0] = ctx->ybuf[0];
                a.ybuf[1] = ctx->ybuf[1];
                a.u = op->kind == LX_OP_BURGERS2D ? scratch + static_cast<size_t>(K) * N : nullptr;
                a.u32 = ctx->u32;
                for (int k = 0; k < K; ++k) {
                    a.p[k] = scratch + static_cast<size_t>(k) * N;
                    a.p2[k] = ctx->blk_ws[k];
                }
                a.coef = ctx->coef;
                a.xi = ctx->xi;
                s = ensure_partials(ctx, 2 * static_cast<size_t>(depth) * a.nb * (1 + K));
                if (s != LX_OK) return cleanup(s);
                a.partials = ctx->partials;
                a.ctl = ctx->ctl;
                if (hipMemcpyAsync(ctx->ctl, &init, sizeof(LoopCtl), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
                    return cleanup(fail(ctx, LX_EDEVICE, "state upload failed"));
                const int n = std::max(1, sweeps / depth);
                hipError_t e = hipSuccess;
                for (int L = 0; L < 2 && e == hipSuccess; ++L)
                    e = lx::launch_leja_stream(opcode, K, depth, fp32, a, L, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ctx->tev[0], ctx->stream);
                for (int L = 2; L < n + 2 && e == hipSuccess; ++L)
                    e = lx::launch_leja_stream(opcode, K, depth, fp32, a, L, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ctx->tev[1], ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(ctx->tev[1]);
                if (e != hipSuccess)
                    return cleanup(fail(ctx, LX_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e)));
                const double us = elapsed(ctx->tev[0], ctx->tev[1]) * 1e3 / (static_cast<double>(depth) * n);
                char line[112];
                std::snprintf(line, sizeof(line), "%d 64 1 %d 2 %d %.3f\n", 100 + depth, g.bands, a.nb, us);
                rep += line;
                if (us < best_pair_us) {
                    best_pair_us = us;
                    best.depth = depth;
                    best.stream = 1;
                    best.bands = bands == g0.bands ? 0 : bands;
                    best.snb = 0;
                }
            }
        }
        if (!(best_pair_us < best_us)) {
            best.depth = 1;
            best.stream = 0;
        }
    }
    const double best_iter_us = std::min(best_us, best_pair_us);
    ctx->tuned[std::make_tuple(op->kind, nx, ny, K, op->prec)] = best;
    if (report != nullptr && report_len > 0) {
        std::snprintf(report, report_len, "%s", rep.c_str());
    }
    const char* path = std::getenv("LX_TUNE_CACHE");
    if (path != nullptr && *path != 0) {
        FILE* f = std::fopen(path, "a");
        if (f != nullptr) {
            std::fprintf(f,
                         "{\"kind\": %d, \"nx\": %d, \"ny\": %d, \"K\": %d, \"prec\": %d, \"tx\": %d, "
                         "\"ty\": %d, \"ry\": %d, \"vec\": %d, \"nb\": %d, \"depth\": %d, \"th\": %d, "
                         "\"pnb\": %d, \"stream\": %d, \"bands\": %d, \"snb\": %d, \"us\": %.3f}\n",
                         op->kind, nx, ny, K, op->prec, best.tx, best.ty, best.ry, best.vec, best.nb, best.depth,
                         best.th, best.pnb, best.stream, best.bands, best.snb, best_iter_us);
            std::fclose(f);
        }
    }
    return cleanup(LX_OK);
}

lx_status lx_bandwidth_probe(lx_ctx* ctx, int kind, size_t n, int reps, double* gbs) {
    if (ctx == nullptr || gbs == nullptr) return LX_EINVAL;
    if ((kind != 0 && kind != 1) || n < 2 || n % 2 != 0 || reps < 1)
        return fail(ctx, LX_EINVAL, "probe kind %d, n %zu, reps %d", kind, n, reps);
    double* buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * n * 3) != hipSuccess) return fail(ctx, LX_ENOMEM, "probe vectors");
    auto cleanup = [&](lx_status r) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(buf);
        return r;
    };
    lx_status s = ensure_timing_events(ctx, 2);
    if (s != LX_OK) return cleanup(s);
    hipError_t e = hipMemsetAsync(buf, 0, sizeof(double) * n * 3, ctx->stream);
    if (e == hipSuccess) e = lx::launch_probe(kind, buf, buf + n, buf + 2 * n, static_cast<long>(n), ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->tev[0], ctx->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = lx::launch_probe(kind, buf, buf + n, buf + 2 * n, static_cast<long>(n), ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->tev[1], ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ctx->tev[1]);
    if (e != hipSuccess) return cleanup(fail(ctx, LX_EDEVICE, "probe failed: %s", hipGetErrorString(e)));
    const double ms = elapsed(ctx->tev[0], ctx->tev[1]);
    const double bytes = (kind == 0 ? 16.0 : 24.0) * static_cast<double>(n) * reps;
    *gbs = bytes / (ms * 1e-3) / 1e9;
    return cleanup(LX_OK);
}

lx_status lx_leja_points(int M, double* xi) {
    if (xi == nullptr || M < 1 || M > LX_MAX_ITERS + 1) return LX_EINVAL;
    return lx::leja_points(M, xi) ? LX_OK : LX_EINVAL;
}

double lx_phi_scalar(int l, double z) { return lx::phi_scalar(l, z); }

lx_status lx_newton_coeffs(int l, double alpha, double sigma, double h, double c, double gamma, int M, double* d) {
    if (d == nullptr || M < 1 || M > LX_MAX_ITERS + 1 || l < 0 || l > 8) return LX_EINVAL;
    std::vector<double> xi(static_cast<size_t>(M));
    if (!lx::leja_points(M, xi.data())) return LX_EINVAL;
    return lx::newton_coeffs(l, alpha, sigma, h, c, gamma, M, xi.data(), d) ? LX_OK : LX_EINVAL;
}

}  // extern "C"
