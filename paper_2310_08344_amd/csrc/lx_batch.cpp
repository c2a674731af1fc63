// C ABI of batched phi actions (declarations and contracts in lx.h).
//
// Host side: lays out the batch (workgroups per instance in proportion to
// its tiles, partial sums, basis buffers), uploads the descriptors once,
// then enqueues the device pipeline: optional batched power iteration, the
// Newton coefficients of every instance, and the batched sweeps, polled once
// per chunk through a device counter of finished instances.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <string>
#include <vector>

#include "lx.h"
#include "lx_ctx.h"
#include "lx_device.h"
#include "planner.h"
#include "stencil_coeffs.h"

using lx::BatchInst;
using lx::LoopCtl;

namespace {

constexpr long kPointsPerWorkgroup = 16384;   // an instance's share of a launch, per workgroup (default)
constexpr int kMaxWorkgroupsPerInstance = 1024;
constexpr int kFirstChunk = 16;
constexpr int kChunk = 8;
constexpr size_t kBatchGraphs = 4;            // captured pipelines kept per context

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

// The class of a batch for the tuned launch shapes: whether any instance
// is a Burgers Jacobian, then its distinct grid sides.
std::vector<int> batch_class(int n, const lx_instance* inst) {
    bool burgers = false;
    std::vector<std::pair<int, int>> sides;
    for (int i = 0; i < n; ++i) {
        burgers = burgers || inst[i].op.kind == LX_OP_BURGERS2D;
        sides.emplace_back(inst[i].op.nx, inst[i].op.ny);
    }
    std::sort(sides.begin(), sides.end());
    sides.erase(std::unique(sides.begin(), sides.end()), sides.end());
    std::vector<int> key{burgers ? 1 : 0};
    for (const auto& q : sides) {
        key.push_back(q.first);
        key.push_back(q.second);
    }
    return key;
}

void drop_graphs(lx_batch_ws& W) {
    for (auto& g : W.graphs)
        if (g.exec != nullptr) (void)hipGraphExecDestroy(g.exec);
    W.graphs.clear();
}

}  // namespace

// frees the batch workspaces (called by lx_destroy)
void lx_internal_free_batch(lx_ctx* ctx) {
    lx_batch_ws& b = ctx->batch;
    drop_graphs(b);
    if (b.cap_stream != nullptr) (void)hipStreamDestroy(b.cap_stream);
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

extern "C" lx_status lx_set_batch_graphs(lx_ctx* ctx, int on) {
    if (ctx == nullptr) return LX_EINVAL;
    if (on != 0 && on != 1) return lx_internal_fail(ctx, LX_EINVAL, "lx_set_batch_graphs: on must be 0 or 1");
    ctx->batch.use_graphs = on;
    if (!on) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess)
            return lx_internal_fail(ctx, LX_EDEVICE, "stream synchronisation failed");
        drop_graphs(ctx->batch);
    }
    return LX_OK;
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
    // the tuned shape of this batch class (lx_tune_batched), unless
    // lx_set_depth forces the iterations per launch
    lx::BatchShape ts{};
    if (ctx->depth_forced == 0) {
        auto it = ctx->batch.tuned.find(batch_class(n, inst));
        if (it != ctx->batch.tuned.end()) ts = it->second;
    }
    const int want_depth = ctx->depth_forced != 0 ? ctx->depth_forced : ts.depth;
    bool pair = want_depth != 1;
    bool blk = want_depth != 1 && want_depth != 2;
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
    int th = (ctx->pair_th == 8 || ctx->pair_th == 16) ? ctx->pair_th
             : (ts.th == 8 || ts.th == 16)               ? ts.th
                                                          : (any_burgers ? 8 : 16);
    if (blk && any_burgers) th = 8;   // the Burgers window layout takes 8-row tiles in a batch
    const long ppw = ts.ppw > 0 ? ts.ppw : kPointsPerWorkgroup;
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
        const int tpw = static_cast<int>(std::max(1L, ppw / tile_points));
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
    const void* addr_before[] = {W.d_inst, W.d_ctl, W.d_block_inst, W.d_coef, W.d_partials, W.d_basis, W.d_done};
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
    {
        // a captured pipeline holds the workspace addresses: drop every one
        // once a workspace has moved
        const void* addr_after[] = {W.d_inst, W.d_ctl, W.d_block_inst, W.d_coef, W.d_partials, W.d_basis, W.d_done};
        if (!std::equal(std::begin(addr_before), std::end(addr_before), std::begin(addr_after))) drop_graphs(W);
    }

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
    }
    const int last = blk ? (max_budget + BD - 1) / BD + 2 : (pair ? (max_budget + 1) / 2 + 1 : max_budget);
    const int per = blk ? BD : (pair ? 2 : 1);
    // the device pipeline: spectral bounds (Listing 7), Newton coefficients,
    // then window (or one- or two-iteration) launches first .. first+count-1
    auto enqueue_head = [&](hipStream_t q) -> hipError_t {
        hipError_t e = hipSuccess;
        if (power_iters > 0) {
            e = lx::launch_batch_fill_x0(d_inst, W.d_block_inst, total_blocks, q);
            if (e == hipSuccess) e = lx::launch_batch_power_norm(d_inst, W.d_block_inst, total_blocks, W.d_partials, q);
            for (int k = 0; k < power_iters && e == hipSuccess; ++k)
                e = lx::launch_batch_power_sweep(d_inst, W.d_block_inst, total_blocks, W.d_partials, k, q);
            if (e == hipSuccess)
                e = lx::launch_batch_power_final(d_inst, n, W.d_partials, power_iters - 1, safety, q);
        }
        if (e == hipSuccess) e = lx::launch_batch_coeffs(d_inst, n, ctx->xi, W.d_coef, ld, q);
        return e;
    };
    auto enqueue_loop = [&](hipStream_t q, int first, int count) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int L = first; L < first + count && e == hipSuccess; ++L) {
            if (blk) {
                e = lx::launch_batch_block(d_inst, d_ctl, W.d_block_inst, total_blocks, any_burgers, th, W.d_partials,
                                           W.d_coef, ld, ctx->xi, W.d_done, L, q);
            } else if (pair) {
                e = lx::launch_batch_pair(d_inst, d_ctl, W.d_block_inst, total_blocks, any_burgers, th, W.d_partials,
                                          W.d_coef, ld, ctx->xi, W.d_done, L, q);
            } else {
                e = lx::launch_batch_sweep(d_inst, d_ctl, W.d_block_inst, total_blocks, W.d_partials, W.d_coef, ld,
                                           ctx->xi, W.d_done, L, q);
            }
        }
        return e;
    };
    // what a captured pipeline bakes in: sizes, launch shape and addresses
    std::vector<long long> key{n, total_blocks, blk ? 1 : 0, pair ? 1 : 0, th, any_burgers ? 1 : 0, power_iters,
                               ld, static_cast<long long>(ppw)};
    {
        long long sb;
        std::memcpy(&sb, &safety, sizeof(sb));
        key.push_back(sb);
        for (const void* a : {static_cast<const void*>(d_inst), static_cast<const void*>(d_ctl),
                              static_cast<const void*>(W.d_block_inst), static_cast<const void*>(W.d_partials),
                              static_cast<const void*>(W.d_coef), static_cast<const void*>(W.d_done),
                              static_cast<const void*>(ctx->xi)})
            key.push_back(static_cast<long long>(reinterpret_cast<uintptr_t>(a)));
    }
    ++W.calls;
    lx_batch_graph* graph = nullptr;
    if (W.use_graphs && !timing) {
        for (auto& g : W.graphs)
            if (g.key == key) graph = &g;
    }

    int launched = 0, chunk_id = 0, last_slot = 0;
    bool finished = false;
    const bool replayed = graph != nullptr;
    if (graph != nullptr) {
        // one captured pipeline, then one look at the finished count; a batch
        // that needs more launches than were captured goes on chunk by chunk
        graph->last_use = W.calls;
        LXB_HIP(ctx, hipGraphLaunch(graph->exec, st));
        launched = graph->launches;
        LXB_HIP(ctx, hipMemcpyAsync(&W.h_done[0], W.d_done, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        LXB_HIP(ctx, hipEventRecord(ctx->poll_ev[0], st));
        LXB_HIP(ctx, hipEventSynchronize(ctx->poll_ev[0]));
        finished = W.h_done[0] >= static_cast<unsigned>(n) || launched > last;
        chunk_id = 1;
    } else {
        if (timing) LXB_HIP(ctx, hipEventRecord(ctx->tev[0], st));
        LXB_HIP(ctx, enqueue_head(st));
        if (timing) LXB_HIP(ctx, hipEventRecord(ctx->tev[1], st));
    }

    // ---- batched sweeps (one or two iterations, or a window, per launch) ----
    // windows: at most ceil(budget / depth) windows, one re-execution (one
    // output) and one publishing launch per instance
    const int first_chunk = std::max(3, kFirstChunk / per), next_chunk = std::max(2, kChunk / per);
    int chunk = graph != nullptr ? next_chunk : first_chunk;
    while (!finished && launched <= last) {
        const int cnt = std::min(chunk, last + 1 - launched);
        LXB_HIP(ctx, enqueue_loop(st, launched, cnt));
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

    // ---- capture the windows pipeline for later calls with this layout ----
    // as many window launches as this call needed (every instance's working
    // launches and the one that publishes it); a replay that needed more
    // than it holds is captured again.
    if (blk && W.use_graphs && !timing) {
        int needed = 1;
        for (int i = 0; i < n; ++i) needed = std::max(needed, h_ctl[i].slot[2].n_work + 1);
        needed = std::min(needed, last + 1);
        if (graph != nullptr && needed > graph->launches) {
            (void)hipGraphExecDestroy(graph->exec);
            W.graphs.erase(W.graphs.begin() + (graph - W.graphs.data()));
            graph = nullptr;
        }
        if (graph == nullptr) {
            // a failed capture leaves the layout uncaptured; the call's results stand
            if (W.cap_stream == nullptr && hipStreamCreateWithFlags(&W.cap_stream, hipStreamNonBlocking) != hipSuccess)
                W.cap_stream = nullptr;
            hipGraph_t g = nullptr;
            if (W.cap_stream != nullptr &&
                hipStreamBeginCapture(W.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                hipError_t e = enqueue_head(W.cap_stream);
                if (e == hipSuccess) e = enqueue_loop(W.cap_stream, 0, needed);
                const hipError_t e2 = hipStreamEndCapture(W.cap_stream, &g);
                hipGraphExec_t ex = nullptr;
                if (e == hipSuccess && e2 == hipSuccess && g != nullptr &&
                    hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
                    if (W.graphs.size() >= kBatchGraphs) {
                        auto lru = std::min_element(W.graphs.begin(), W.graphs.end(),
                                                    [](const lx_batch_graph& a, const lx_batch_graph& b) {
                                                        return a.last_use < b.last_use;
                                                    });
                        (void)hipGraphExecDestroy(lru->exec);
                        W.graphs.erase(lru);
                    }
                    W.graphs.push_back(lx_batch_graph{key, ex, needed, W.calls});
                }
                if (g != nullptr) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
            }
        }
    }
    S.batch_graph = replayed ? 1 : 0;
    if (worst != LX_OK) ctx->err = "at least one instance did not converge or became non-finite; see its result";
    return worst;
}

// Times the batch itself under every candidate launch shape and keeps the
// fastest for its class (lx.h).
extern "C" lx_status lx_tune_batched(lx_ctx* ctx, int n, const lx_instance* inst, int power_iters, double safety,
                                     const lx_leja_opts* o, int repeats, char* report, size_t report_len) {
    if (ctx == nullptr) return LX_EINVAL;
    if (n < 1 || n > 65536 || inst == nullptr) return lx_internal_fail(ctx, LX_EINVAL, "tune: batch of %d instances", n);
    if (repeats < 1 || repeats > 50) return lx_internal_fail(ctx, LX_EINVAL, "tune: repeats %d outside 1..50", repeats);
    bool burgers = false, even = true;
    int min_side = 1 << 30;
    for (int i = 0; i < n; ++i) {
        burgers = burgers || inst[i].op.kind == LX_OP_BURGERS2D;
        even = even && inst[i].op.nx % 2 == 0;
        min_side = std::min(min_side, std::min(inst[i].op.nx, inst[i].op.ny));
    }
    std::vector<lx::BatchShape> cands;
    for (int depth : {lx::kBatchBlockDepth, 2, 1}) {
        if (depth >= 2 && !even) continue;
        if (depth == lx::kBatchBlockDepth && min_side < depth) continue;
        for (int th : {8, 16}) {
            if (depth == 1 && th == 16) continue;                              // th is not used by one sweep
            if (th == 16 && burgers && depth == lx::kBatchBlockDepth) continue;  // windows with Burgers: 8 rows
            for (int ppw : {4096, 8192, 16384, 32768}) cands.push_back(lx::BatchShape{depth, th, ppw});
        }
    }
    const std::vector<int> cls = batch_class(n, inst);
    const int saved_depth = ctx->depth_forced, saved_th = ctx->pair_th;
    ctx->depth_forced = 0;
    ctx->pair_th = 0;
    std::vector<lx_instance_result> res(static_cast<size_t>(n));
    std::string rep;
    double best_ms = 1e300;
    lx::BatchShape best{};
    lx_status status = LX_OK;
    for (const lx::BatchShape& c : cands) {
        ctx->batch.tuned[cls] = c;
        std::vector<double> ms;
        for (int r = 0; r <= repeats && status == LX_OK; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            const lx_status s = lx_phi_leja_batched(ctx, n, inst, power_iters, safety, o, res.data());
            const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (s != LX_OK && s != LX_ENOTCONV) status = s;
            if (r > 0) ms.push_back(t);   // the first call is a warm-up (and captures the pipeline)
        }
        if (status != LX_OK) break;
        std::sort(ms.begin(), ms.end());
        const double med = ms[ms.size() / 2];
        char line[96];
        std::snprintf(line, sizeof(line), "%d %d %d %.4f\n", c.depth, c.th, c.ppw, med);
        rep += line;
        if (med < best_ms) {
            best_ms = med;
            best = c;
        }
    }
    ctx->depth_forced = saved_depth;
    ctx->pair_th = saved_th;
    if (status != LX_OK) {
        ctx->batch.tuned.erase(cls);
        return status;
    }
    ctx->batch.tuned[cls] = best;
    if (report != nullptr && report_len > 0) std::snprintf(report, report_len, "%s", rep.c_str());
    const char* path = std::getenv("LX_TUNE_CACHE");
    if (path != nullptr && *path != 0) {
        FILE* f = std::fopen(path, "a");
        if (f != nullptr) {
            std::fprintf(f, "{\"batch_class\": [");
            for (size_t i = 0; i < cls.size(); ++i) std::fprintf(f, "%s%d", i ? ", " : "", cls[i]);
            std::fprintf(f, "], \"depth\": %d, \"th\": %d, \"ppw\": %d, \"ms\": %.4f}\n", best.depth, best.th, best.ppw,
                         best_ms);
            std::fclose(f);
        }
    }
    return LX_OK;
}

extern "C" lx_status lx_set_batch_shape(lx_ctx* ctx, int n, const lx_instance* inst, int depth, int th, int ppw) {
    if (ctx == nullptr) return LX_EINVAL;
    if (n < 1 || inst == nullptr) return lx_internal_fail(ctx, LX_EINVAL, "batch shape: no instances");
    if (!(depth == 0 || depth == 1 || depth == 2 || depth == lx::kBatchBlockDepth) ||
        !(th == 0 || th == 8 || th == 16) || ppw < 0 || ppw > (1 << 22))
        return lx_internal_fail(ctx, LX_EINVAL, "batch shape: depth %d, th %d, ppw %d", depth, th, ppw);
    const std::vector<int> cls = batch_class(n, inst);
    if (depth == 0 && th == 0 && ppw == 0) ctx->batch.tuned.erase(cls);
    else ctx->batch.tuned[cls] = lx::BatchShape{depth, th, ppw};
    return LX_OK;
}
