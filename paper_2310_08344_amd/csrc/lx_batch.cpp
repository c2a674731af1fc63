// C ABI of batched phi actions (declarations and contracts in lx.h).
//
// Host side: lays out the batch (workgroups per instance in proportion to
// its tiles, partial sums, basis buffers), uploads the descriptors once,
// then enqueues the device pipeline: optional batched power iteration, the
// Newton coefficients of every instance, and the batched sweeps, polled once
// per chunk through a device counter of finished instances.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "lx.h"
#include "lx_ctx.h"
#include "lx_device.h"
#include "planner.h"
#include "stencil_coeffs.h"

using lx::BatchInst;
using lx::LoopCtl;

namespace {

constexpr long kPointsPerWorkgroup = 16384;   // an instance's share of a launch, per workgroup
constexpr int kMaxWorkgroupsPerInstance = 1024;
constexpr int kFirstChunk = 16;
constexpr int kChunk = 8;

#define LXB_HIP(ctx, call)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return lx_internal_fail((ctx), LX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <typename T>
lx_status grow_device(lx_ctx* ctx, T** p, size_t* cap, size_t need) {
    if (need <= *cap) return LX_OK;
    if (*p != nullptr) {
        LXB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    if (hipMalloc(reinterpret_cast<void**>(p), need * sizeof(T)) != hipSuccess)
        return lx_internal_fail(ctx, LX_ENOMEM, "batch workspace of %zu bytes", need * sizeof(T));
    *cap = need;
    return LX_OK;
}

template <typename T>
lx_status grow_pinned(lx_ctx* ctx, T** p, size_t* cap, size_t need) {
    if (need <= *cap) return LX_OK;
    if (*p != nullptr) {
        LXB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipHostFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(p), need * sizeof(T), hipHostMallocDefault) != hipSuccess)
        return lx_internal_fail(ctx, LX_ENOMEM, "pinned batch staging of %zu bytes", need * sizeof(T));
    *cap = need;
    return LX_OK;
}

}  // namespace

// frees the batch workspaces (called by lx_destroy)
void lx_internal_free_batch(lx_ctx* ctx) {
    lx_batch_ws& b = ctx->batch;
    (void)hipFree(b.d_inst);
    (void)hipFree(b.d_ctl);
    (void)hipFree(b.d_block_inst);
    (void)hipFree(b.d_coef);
    (void)hipFree(b.d_partials);
    (void)hipFree(b.d_basis);
    (void)hipFree(b.d_done);
    (void)hipHostFree(b.h_inst);
    (void)hipHostFree(b.h_ctl);
    (void)hipHostFree(b.h_block_inst);
    (void)hipHostFree(b.h_done);
    (void)hipFree(b.d_feat);
    (void)hipHostFree(b.h_feat);
    b = lx_batch_ws{};
}

extern "C" lx_status lx_phi_leja_batched(lx_ctx* ctx, int n, const lx_instance* inst, int power_iters,
                                         double safety, const lx_leja_opts* o, lx_instance_result* res) {
    if (ctx == nullptr) return LX_EINVAL;
    ctx->stats = lx_stats{};
    if (n < 1 || n > 65536 || inst == nullptr || res == nullptr)
        return lx_internal_fail(ctx, LX_EINVAL, "batch of %d instances (1..65536) with inputs and results", n);
    if (power_iters < 0 || power_iters > LX_MAX_ITERS)
        return lx_internal_fail(ctx, LX_EINVAL, "power_iters %d outside 0..%d", power_iters, LX_MAX_ITERS);
    if (power_iters > 0 && (!(safety > 0.0) || !std::isfinite(safety)))
        return lx_internal_fail(ctx, LX_EINVAL, "safety must be finite and > 0");
    lx_leja_opts opt{1e-8, 0.0, 500, 1e4};
    if (o != nullptr) opt = *o;
    if (!(opt.rtol >= 0.0) || !(opt.atol >= 0.0) || !std::isfinite(opt.rtol) || !std::isfinite(opt.atol))
        return lx_internal_fail(ctx, LX_EINVAL, "tolerances must be finite and >= 0");
    if (opt.max_iters < 1 || opt.max_iters > LX_MAX_ITERS)
        return lx_internal_fail(ctx, LX_EINVAL, "max_iters %d outside 1..%d", opt.max_iters, LX_MAX_ITERS);

    // ---- layout ----
    // two iterations per launch when every instance allows 16-byte pairs;
    // windows of kBatchBlockDepth when, moreover, every side reaches the
    // window's halo and lx_set_depth does not ask for one or two
    constexpr int BD = lx::kBatchBlockDepth;
    bool pair = ctx->depth_forced != 1;
    bool blk = ctx->depth_forced != 1 && ctx->depth_forced != 2;
    bool any_burgers = false;
    for (int i = 0; i < n; ++i) {
        const lx_instance& q = inst[i];
        any_burgers = any_burgers || q.op.kind == LX_OP_BURGERS2D;
        pair = pair && q.op.nx % 2 == 0 && aligned16(q.d_v) && aligned16(q.d_out) &&
               (q.d_u == nullptr || aligned16(q.d_u)) && (q.d_x0 == nullptr || aligned16(q.d_x0));
        blk = blk && q.op.nx >= BD && q.op.ny >= BD;
    }
    blk = blk && pair;
    if (blk) pair = false;
    // tile rows: 16 (40 KB of LDS, 4 workgroups per CU) unless the Burgers
    // state needs room too, then 8 (36 KB)
    int th = (ctx->pair_th == 8 || ctx->pair_th == 16) ? ctx->pair_th : (any_burgers ? 8 : 16);
    if (blk && any_burgers) th = 8;   // the Burgers window layout takes 8-row tiles in a batch
    std::vector<BatchInst> hi(static_cast<size_t>(n));
    std::vector<int> budget(static_cast<size_t>(n));
    int total_blocks = 0, max_budget = 1;
    long part_total = 0;
    size_t basis_total = 0;
    for (int i = 0; i < n; ++i) {
        const lx_instance& q = inst[i];
        lx_status s = lx_internal_check_op(ctx, &q.op, static_cast<size_t>(1) << 40);
        if (s != LX_OK) return lx_internal_fail(ctx, s, "instance %d: %s", i, lx_last_error(ctx));
        if (q.op.prec != LX_FP64) return lx_internal_fail(ctx, LX_EINVAL, "instance %d: batches run in FP64", i);
        if (q.op.kind != LX_OP_DIFFADV2D && q.op.kind != LX_OP_BURGERS2D)
            return lx_internal_fail(ctx, LX_EINVAL, "instance %d: batches take the five-point operators", i);
        if (q.d_v == nullptr || q.d_out == nullptr || q.d_out == q.d_v)
            return lx_internal_fail(ctx, LX_EINVAL, "instance %d: needs distinct d_v and d_out", i);
        if (q.op.kind == LX_OP_BURGERS2D && q.d_u == nullptr)
            return lx_internal_fail(ctx, LX_EINVAL, "instance %d: Burgers Jacobian needs d_u", i);
        if (q.l < 0 || q.l > 8) return lx_internal_fail(ctx, LX_EINVAL, "instance %d: l = %d outside 0..8", i, q.l);
        if (!(q.h > 0.0) || !std::isfinite(q.h)) return lx_internal_fail(ctx, LX_EINVAL, "instance %d: h", i);
        if (power_iters == 0 && (!(q.c <= 0.0) || !(q.gamma > 0.0) || !std::isfinite(q.c) || !std::isfinite(q.gamma)))
            return lx_internal_fail(ctx, LX_EINVAL, "instance %d: c <= 0 and gamma > 0 required", i);
        if (q.budget < 0 || q.budget > opt.max_iters)
            return lx_internal_fail(ctx, LX_EINVAL, "instance %d: budget %d outside 0..max_iters", i, q.budget);
        BatchInst& b = hi[static_cast<size_t>(i)];
        std::memset(&b, 0, sizeof(b));
        b.kind = q.op.kind == LX_OP_DIFFADV2D ? lx::kOpDiffAdv : lx::kOpBurgersJ;
        b.nx = q.op.nx;
        b.ny = q.op.ny;
        const bool al = aligned16(q.d_v) && aligned16(q.d_out) && (q.d_u == nullptr || aligned16(q.d_u)) &&
                        (q.d_x0 == nullptr || aligned16(q.d_x0));
        b.vec = (al && b.nx % 2 == 0) ? 2 : 1;
        b.l = q.l;
        long tile_points;
        if (pair || blk) {
            b.tiles_x = (b.nx + 127) / 128;
            b.tiles_y = (b.ny + th - 1) / th;
            tile_points = 128L * th;
        } else {
            b.tiles_x = (b.nx + lx::kBatchTx * b.vec - 1) / (lx::kBatchTx * b.vec);
            b.tiles_y = (b.ny + lx::kBatchTy - 1) / lx::kBatchTy;
            tile_points = static_cast<long>(lx::kBatchTx) * b.vec * lx::kBatchTy;
        }
        b.ptiles_x = (b.nx + lx::kBatchTx * b.vec - 1) / (lx::kBatchTx * b.vec);
        b.ptiles_y = (b.ny + lx::kBatchTy * lx::kBatchPowerRows - 1) / (lx::kBatchTy * lx::kBatchPowerRows);
        const int T = b.tiles_x * b.tiles_y;
        const int tpw = static_cast<int>(std::max(1L, kPointsPerWorkgroup / tile_points));
        b.nb = std::min(std::max((T + tpw - 1) / tpw, 1), kMaxWorkgroupsPerInstance);
        b.wg_begin = total_blocks;
        total_blocks += b.nb;
        b.part_off = part_total;
        part_total += (blk ? 4L * BD : (pair ? 8L : 4L)) * b.nb;   // [2][nb][NV] partial sums
        b.has_x0 = q.d_x0 != nullptr;
        b.dx = q.op.dx;
        b.dy = q.op.dy;
        b.D = q.op.D;
        b.vx = q.op.vx;
        b.vy = q.op.vy;
        b.nu = q.op.nu;
        b.h = q.h;
        b.c = q.c;
        b.gamma = q.gamma;
        const int sk = b.kind == lx::kOpDiffAdv ? 0 : 1;
        lx::stencil_coeffs(sk, b.dx, b.dy, b.D, b.vx, b.vy, b.nu, 0.0, 1.0, b.pw);
        if (power_iters == 0) lx::stencil_coeffs(sk, b.dx, b.dy, b.D, b.vx, b.vy, b.nu, b.c, b.gamma, b.st);
        b.u = q.op.kind == LX_OP_BURGERS2D ? q.d_u : nullptr;
        b.v = q.d_v;
        b.out = q.d_out;
        b.x0 = q.d_x0;
        basis_total += (blk ? 3 : 2) * static_cast<size_t>(b.nx) * b.ny;   // windows: a second output buffer
        budget[static_cast<size_t>(i)] = q.budget > 0 ? q.budget : opt.max_iters;
        max_budget = std::max(max_budget, budget[static_cast<size_t>(i)]);
    }
    if (total_blocks > (1 << 30)) return lx_internal_fail(ctx, LX_EINVAL, "batch too large");
    const int ld = max_budget + (blk ? BD + 1 : (pair ? 2 : 1));   // Newton coefficients per instance

    // ---- workspaces ----
    lx_batch_ws& W = ctx->batch;
    lx_status s = LX_OK;
    const size_t nn = static_cast<size_t>(n), nblk = static_cast<size_t>(total_blocks);
    if ((s = grow_device(ctx, reinterpret_cast<BatchInst**>(&W.d_inst), &W.cap_d_inst, nn)) != LX_OK ||
        (s = grow_device(ctx, reinterpret_cast<LoopCtl**>(&W.d_ctl), &W.cap_d_ctl, nn)) != LX_OK ||
        (s = grow_pinned(ctx, reinterpret_cast<BatchInst**>(&W.h_inst), &W.cap_h_inst, nn)) != LX_OK ||
        (s = grow_pinned(ctx, reinterpret_cast<LoopCtl**>(&W.h_ctl), &W.cap_h_ctl, nn)) != LX_OK ||
        (s = grow_device(ctx, &W.d_block_inst, &W.cap_d_blk, nblk)) != LX_OK ||
        (s = grow_pinned(ctx, &W.h_block_inst, &W.cap_h_blk, nblk)) != LX_OK ||
        (s = grow_device(ctx, &W.d_coef, &W.cap_coef, nn * ld)) != LX_OK ||
        (s = grow_device(ctx, &W.d_partials, &W.cap_partials, static_cast<size_t>(part_total))) != LX_OK ||
        (s = grow_device(ctx, &W.d_basis, &W.cap_basis, basis_total)) != LX_OK ||
        (s = grow_device(ctx, &W.d_done, &W.cap_done, 1)) != LX_OK ||
        (s = grow_pinned(ctx, &W.h_done, &W.cap_h_done, 2)) != LX_OK)
        return s;
    s = lx_internal_ensure_xi(ctx, ld);
    if (s != LX_OK) return s;

    // ---- descriptors ----
    BatchInst* h_inst = static_cast<BatchInst*>(W.h_inst);
    LoopCtl* h_ctl = static_cast<LoopCtl*>(W.h_ctl);
    size_t boff = 0;
    for (int i = 0; i < n; ++i) {
        BatchInst b = hi[static_cast<size_t>(i)];
        const size_t N = static_cast<size_t>(b.nx) * b.ny;
        b.y[0] = W.d_basis + boff;
        b.y[1] = W.d_basis + boff + N;
        boff += 2 * N;
        b.out2 = nullptr;
        if (blk) {
            b.out2 = W.d_basis + boff;
            boff += N;
        }
        h_inst[i] = b;
        for (int k = 0; k < b.nb; ++k) W.h_block_inst[b.wg_begin + k] = i;
        LoopCtl& c = h_ctl[i];
        std::memset(&c, 0, sizeof(c));
        c.rtol = opt.rtol;
        c.atol = opt.atol;
        c.fp32_switch = -1.0;
        c.max_iters = budget[static_cast<size_t>(i)];
        c.slot[0].active[0] = 1;
        c.slot[0].iters[0] = c.max_iters;
    }
    W.h_done[0] = 0u;
    hipStream_t st = ctx->stream;
    BatchInst* d_inst = static_cast<BatchInst*>(W.d_inst);
    LoopCtl* d_ctl = static_cast<LoopCtl*>(W.d_ctl);
    LXB_HIP(ctx, hipMemcpyAsync(d_inst, h_inst, sizeof(BatchInst) * n, hipMemcpyHostToDevice, st));
    LXB_HIP(ctx, hipMemcpyAsync(d_ctl, h_ctl, sizeof(LoopCtl) * n, hipMemcpyHostToDevice, st));
    LXB_HIP(ctx, hipMemcpyAsync(W.d_block_inst, W.h_block_inst, sizeof(int) * total_blocks, hipMemcpyHostToDevice, st));
    LXB_HIP(ctx, hipMemcpyAsync(W.d_done, W.h_done, sizeof(unsigned), hipMemcpyHostToDevice, st));

    const bool timing = ctx->timing != 0;
    if (timing) {
        s = lx_internal_ensure_timing_events(ctx, 4);
        if (s != LX_OK) return s;
        LXB_HIP(ctx, hipEventRecord(ctx->tev[0], st));
    }
    // ---- spectral bounds (Listing 7) ----
    if (power_iters > 0) {
        LXB_HIP(ctx, lx::launch_batch_fill_x0(d_inst, W.d_block_inst, total_blocks, st));
        LXB_HIP(ctx, lx::launch_batch_power_norm(d_inst, W.d_block_inst, total_blocks, W.d_partials, st));
        for (int k = 0; k < power_iters; ++k)
            LXB_HIP(ctx, lx::launch_batch_power_sweep(d_inst, W.d_block_inst, total_blocks, W.d_partials, k, st));
        LXB_HIP(ctx, lx::launch_batch_power_final(d_inst, n, W.d_partials, power_iters - 1, safety, st));
    }
    // ---- Newton coefficients on the device ----
    LXB_HIP(ctx, lx::launch_batch_coeffs(d_inst, n, ctx->xi, W.d_coef, ld, st));
    if (timing) LXB_HIP(ctx, hipEventRecord(ctx->tev[1], st));

    // ---- batched sweeps (one or two iterations, or a window, per launch) ----
    // windows: at most ceil(budget / depth) windows, one re-execution (one
    // output) and one publishing launch per instance
    const int last = blk ? (max_budget + BD - 1) / BD + 2 : (pair ? (max_budget + 1) / 2 + 1 : max_budget);
    const int per = blk ? BD : (pair ? 2 : 1);
    int launched = 0, chunk_id = 0, last_slot = 0;
    const int first_chunk = std::max(3, kFirstChunk / per), next_chunk = std::max(2, kChunk / per);
    int chunk = first_chunk;
    while (launched <= last) {
        const int cnt = std::min(chunk, last + 1 - launched);
        for (int i = 0; i < cnt; ++i) {
            if (blk) {
                LXB_HIP(ctx, lx::launch_batch_block(d_inst, d_ctl, W.d_block_inst, total_blocks, any_burgers, th,
                                                    W.d_partials, W.d_coef, ld, ctx->xi, W.d_done, launched + i, st));
            } else if (pair) {
                LXB_HIP(ctx, lx::launch_batch_pair(d_inst, d_ctl, W.d_block_inst, total_blocks, any_burgers, th,
                                                   W.d_partials, W.d_coef, ld, ctx->xi, W.d_done, launched + i, st));
            } else {
                LXB_HIP(ctx, lx::launch_batch_sweep(d_inst, d_ctl, W.d_block_inst, total_blocks, W.d_partials,
                                                    W.d_coef, ld, ctx->xi, W.d_done, launched + i, st));
            }
        }
        launched += cnt;
        const int slot = chunk_id & 1;
        LXB_HIP(ctx, hipMemcpyAsync(&W.h_done[slot], W.d_done, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        LXB_HIP(ctx, hipEventRecord(ctx->poll_ev[slot], st));
        last_slot = slot;
        if (chunk_id >= 1) {
            const int prev = slot ^ 1;
            LXB_HIP(ctx, hipEventSynchronize(ctx->poll_ev[prev]));
            if (W.h_done[prev] >= static_cast<unsigned>(n)) break;
        }
        ++chunk_id;
        chunk = next_chunk;
    }
    if (timing) LXB_HIP(ctx, hipEventRecord(ctx->tev[2], st));
    LXB_HIP(ctx, hipEventSynchronize(ctx->poll_ev[last_slot]));
    LXB_HIP(ctx, hipMemcpyAsync(h_ctl, d_ctl, sizeof(LoopCtl) * n, hipMemcpyDeviceToHost, st));
    LXB_HIP(ctx, hipMemcpyAsync(h_inst, d_inst, sizeof(BatchInst) * n, hipMemcpyDeviceToHost, st));
    LXB_HIP(ctx, hipStreamSynchronize(st));

    // ---- results ----
    lx_stats& S = ctx->stats;
    lx_status worst = LX_OK;
    double bytes = 0.0;
    int max_iter = 0;
    for (int i = 0; i < n; ++i) {
        const lx::SweepState& f = h_ctl[i].slot[2];
        lx_instance_result& r = res[i];
        const BatchInst& b = h_inst[i];
        r.status = f.done ? f.status : LX_EDEVICE;
        r.fallback = 0;
        r.iters = f.iters[0];
        r.err = f.err[0];
        r.pnorm = f.pnorm[0];
        r.rho_hat = power_iters > 0 ? b.rho : 0.0;
        r.c = b.c;
        r.gamma = b.gamma;
        if (r.status == LX_ENONFINITE || r.status == LX_EDEVICE) worst = static_cast<lx_status>(r.status);
        else if (r.status == LX_ENOTCONV && worst == LX_OK) worst = LX_ENOTCONV;
        const double N = static_cast<double>(b.nx) * b.ny;
        const double ub = b.kind == lx::kOpBurgersJ ? 8.0 : 0.0;
        if (blk) {
            // counted on the device by the launches that did work
            bytes += N * f.bytes_pp;
            max_iter = std::max(max_iter, f.n_levels);
        } else if (pair) {
            // launches 0..F-1 ran both sweeps (launch 0 writes p without
            // reading it), an even final test added a flush of the deferred term
            const int F = (f.iter + 1) / 2;
            bytes += N * (24.0 + ub);
            for (int L = 1; L < F; ++L) bytes += N * (16.0 + ub + (f.iters[0] >= 2 * L ? 16.0 : 0.0));
            if (f.iter % 2 == 0) bytes += N * 24.0;
            max_iter = std::max(max_iter, 2 * F);
        } else {
            // sweep 0 reads v, writes y_1 and p; later sweeps read y and p, write both
            bytes += N * ((24.0 + ub) + (32.0 + ub) * std::max(f.iter - 1, 0));
            max_iter = std::max(max_iter, f.iter);
        }
        bytes += N * (16.0 + ub) * power_iters;
    }
    S.n_apply = max_iter;
    S.depth = per;
    S.bytes = bytes;
    if (timing) {
        S.plan_ms = lx_internal_elapsed(ctx->tev[0], ctx->tev[1]);
        S.loop_ms = lx_internal_elapsed(ctx->tev[1], ctx->tev[2]);
        S.sweep_ms = lx_internal_elapsed(ctx->tev[0], ctx->tev[2]);
    }
    S.status = worst;
    if (worst != LX_OK) ctx->err = "at least one instance did not converge or became non-finite; see its result";
    return worst;
}
