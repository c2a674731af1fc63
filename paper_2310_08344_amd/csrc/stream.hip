// Windows of D Leja iterations per launch by register streaming (gfx950),
// FP64, for the five-point diffusion-advection operator; and power
// iteration with many sweeps per launch in the same way.
//
// The window semantics are those of leja_block (window_device.h): every
// output takes the one-iteration loop's terms in the same order, and the
// stop rule (Sec. 2.2) is applied at every term m+1 .. m+D from the sums of
// squares the window records.  Only the way the levels are formed differs.
//
// Every wavefront works alone on an item: a strip of 128 columns (64 lanes,
// a column pair each) and a band of rows, marched from top to bottom with no
// LDS and no barrier.  Its 128 columns are the item's output columns and D
// columns on each side; level j (the basis vector y_{m+j}) is valid on the
// strip minus j columns on each side, so after D levels the output columns
// remain.  Rows are staged from D above the band to D below it.  At step t
// the wavefront loads row t of y_m (level 0) and then forms level j at row
// t - j for j = 1..D from the two rows of level j-1 it kept in registers and
// the row of level j-1 it just formed (the Newton recurrence of Sec. 2.1,
// Eq. (2)).  The side neighbours of a column pair come from the neighbouring
// lanes (DPP wavefront shifts).  An output row enters the registers when
// level 0 reaches it, takes term j when level j does, and leaves after its
// last term: D + 1 rows of every output are in flight.  Nothing is formed
// twice along y (the LDS-tile kernel forms up to 1.7 points per output point
// at D = 6 on 8-row tiles); along x the strip's side columns are formed by
// two wavefronts (128 columns per 128 - 2D outputs).
//
// Each wavefront's items are a contiguous run of bands of one XCD, so the
// side columns a neighbouring strip also loads come from that XCD's L2.
#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"
#include "tile_device.h"
#include "window_device.h"

namespace lx {
namespace {

using namespace dev;

constexpr int kStreamWaves = kBlockThreads / 64;   // wavefronts per workgroup, each on its own items

// Columns [xs, xs + ws) and rows [yb, yb + hb) of item i: items are numbered
// band-major over sx strips and by bands; strip widths are even.
struct StreamItem {
    int xs, ws, yb, hb;
};

__device__ __forceinline__ StreamItem stream_geom(const int i, const int nx, const int ny, const int sx,
                                                  const int by) {
    const int b = i / sx, s = i - b * sx;
    const long half = nx >> 1;
    StreamItem it;
    it.xs = 2 * static_cast<int>((s * half) / sx);
    it.ws = 2 * static_cast<int>(((s + 1) * half) / sx) - it.xs;
    it.yb = static_cast<int>((static_cast<long>(b) * ny) / by);
    it.hb = static_cast<int>((static_cast<long>(b + 1) * ny) / by) - it.yb;
    return it;
}

// This wavefront's index among the a.nb * kStreamWaves of the grid, so that
// the wavefronts of one XCD (workgroup b runs on XCD b % 8) hold a
// contiguous range.
__device__ __forceinline__ int stream_wave(const int wg, const int nb) {
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int slot = (nb >= 8 && (nb & 7) == 0) ? (wg & 7) * (nb >> 3) + (wg >> 3) : wg;
    return slot * kStreamWaves + wave;
}

// The five-point operator of shifted_at, split in two so that a level keeps
// only two rows in registers: stream_partial takes this lane's column pair
// of row C (the side columns from the neighbouring lanes) and the row S
// before it, and forms everything but the last term; stream_complete adds
// the term of the row N after it.  The operand order is stencil_da's:
//   fma(cN, N, fma(cS, S, fma(cE, E, fma(cW, W, cC C)))),
// so every kernel forms the same bits.  All 64 lanes must be active.
__device__ __forceinline__ double2 stream_partial(const Sten& st, const double cc, const double2 S, const double2 C) {
#pragma clang fp contract(off)
    const double w = lane_neighbour<true>(C.y, C.y);    // column j - 1: lane - 1's second column
    const double e = lane_neighbour<false>(C.x, C.x);   // column j + 2: lane + 1's first column
    double2 o;
    o.x = fma(st.c2, S.x, fma(st.c1, C.y, fma(st.c0, w, cc * C.x)));
    o.y = fma(st.c2, S.y, fma(st.c1, e, fma(st.c0, C.x, cc * C.y)));
    // formed here, not where the next step uses it: the neighbour values
    // (convergent cross-lane moves, which stay put) would otherwise be held
    // in registers across the step
    asm volatile("" : "+v"(o.x), "+v"(o.y));
    return o;
}

__device__ __forceinline__ double2 stream_complete(const Sten& st, const double2 q, const double2 N) {
    double2 o;
    o.x = fma(st.c3, N.x, q.x);
    o.y = fma(st.c3, N.y, q.y);
    return o;
}

__device__ __forceinline__ double2 ld_pair(const double* p) { return *reinterpret_cast<const double2*>(p); }

__device__ __forceinline__ double sel(const bool c, const double a, const double b) { return c ? a : b; }

// One item of a window launch (see the file comment).  dk[k][j] = d_{m+j}
// of output k, cc[j-1] the centre coefficient of level j.
//
// Entering step t, lc[j] holds level j at row t-j-1 and lq[j] level j+1 at
// row t-j-1 without its last term; the step completes level j+1 there with
// level j at row t-j, which it has just formed.  Every step forms all D
// levels: before step 2j, level j is formed on rows whose inputs are not all
// staged yet, but such rows only feed rows of higher levels that are
// equally invalid, and no output row is among them (outputs start at row
// D).  A re-execution forms all D levels as well and takes only the terms
// its outputs need.  pr[k][i] holds output k at row t-1-i; slots of rows
// outside the band take no terms and are not stored.  Steps run in pairs,
// which the roles of lc and lq repeat with, so that they stay in place; an
// odd count adds one step past the staged rows that stores nothing.
template <int K, int D>
__device__ __forceinline__ void stream_window_item(const TileArgs<K>& ta, const WindowPlan<K>& w,
                                                   const double (&dk)[K][D + 1], const double (&cc)[D],
                                                   const StreamItem it, const int lane, double (&sy)[D],
                                                   double (&sp)[K][D]) {
    const int nx = ta.nx, ny = ta.ny;
    const int rc = 2 * lane - D;                 // strip column of this lane's pair
    const int gcol = wrap(it.xs + rc, nx);       // even: xs, D and nx are
    const bool ocol = rc >= 0 && rc < it.ws;
    const double mcol = ocol ? 1.0 : 0.0;        // weight of this lane in the sums
    const int T = it.hb + 2 * D;                 // rows staged: the band and D above and below
    const int ytop = it.yb - D;
    const bool first = w.win == 0, store_y = !w.redo;
    const double* __restrict__ yin = w.yin;
    auto row_off = [&](const int t) { return static_cast<long>(wrap(ytop + t, ny)) * nx + gcol; };

    double2 lc[D], lq[D];
    double2 pr[K][D];
#pragma unroll
    for (int j = 0; j < D; ++j) lc[j] = lq[j] = double2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) pr[k][i] = double2{0.0, 0.0};
    // level 0 two rows ahead (T >= 2D >= 2)
    double2 yq0 = ld_pair(yin + row_off(0));
    double2 yq1 = ld_pair(yin + row_off(1));

    for (int t0 = 0; t0 < T; t0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = t0 + u;
            double2 cur = yq0;
            yq0 = yq1;
            yq1 = ld_pair(yin + row_off(t + 2 < T ? t + 2 : T - 1));
            // an output row enters when level 0 reaches it
            double2 pn[K];
            const bool orow = t >= D && t < D + it.hb;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                pn[k].x = dk[k][0] * cur.x;   // p_0 = d_0 y_0 (first window)
                pn[k].y = dk[k][0] * cur.y;
                if (orow && !first && w.nt[k] > 0 && ocol) pn[k] = ld_stream(w.pin[k] + row_off(t));
            }
#pragma unroll
            for (int j = 1; j <= D; ++j) {
                // cur: level j-1 at row t-j+1
                const double2 y = stream_complete(ta.st, lq[j - 1], cur);   // level j at row t-j
                lq[j - 1] = stream_partial(ta.st, cc[j - 1], lc[j - 1], cur);
                lc[j - 1] = cur;
                cur = y;
                // masks as factors, not selects: a select of a product
                // becomes a branch, which splits the step into blocks
                const int r = t - j;
                const bool take = r >= D && r < D + it.hb && j <= w.jmax;
                const double m = take ? mcol : 0.0;
                sy[j - 1] = fma(m, y.x * y.x + y.y * y.y, sy[j - 1]);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool tk = take && w.nt[k] >= j;
                    const double d = tk ? dk[k][j] : 0.0;   // no term: p + 0 y
                    double2& p = pr[k][j - 1];
                    p.x = fma(d, y.x, p.x);
                    p.y = fma(d, y.y, p.y);
                    sp[k][j - 1] = fma(tk ? mcol : 0.0, p.x * p.x + p.y * p.y, sp[k][j - 1]);
                }
            }
            // row t-D is complete: y_{m+D} and every output that took terms
            // (an output that stopped after term j < D has not changed since)
            if (t >= 2 * D && t < T && ocol) {
                const long o = row_off(t - D);
                if (store_y) *reinterpret_cast<double2*>(w.yout + o) = cur;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (w.nt[k] > 0) st_stream(w.pout[k] + o, pr[k][D - 1]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int i = D - 1; i > 0; --i) pr[k][i] = pr[k][i - 1];
                pr[k][0] = pn[k];
            }
        }
    }
}

// Launch L of the window loop: a.tiles_x strips by a.tiles_y bands, a.nb
// workgroups of kStreamWaves wavefronts.
template <int K, int D>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void leja_stream(SweepArgs a,
                                                                                                const int L) {
    if (loop_ended(a.ctl)) return;
    const int wg = static_cast<int>(blockIdx.x);
    WindowPlan<K> w;
    if (!window_enter<kOpDiffAdv, K, D>(a, L, wg, nullptr, w)) return;
    double dk[K][D + 1], cc[D];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int j = 0; j <= D; ++j) dk[k][j] = a.coef[k * a.ld + w.m + j];
#pragma unroll
    for (int j = 0; j < D; ++j) cc[j] = a.aC - a.xi[w.m + j];
    const TileArgs<K> ta = tile_args<kOpDiffAdv, K>(a);
    double sy[D], sp[K][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sy[j] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sp[k][j] = 0.0;
    }
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int items = a.tiles_x * a.tiles_y, G = a.nb * kStreamWaves;
    for (int i = stream_wave(wg, a.nb); i < items; i += G)
        stream_window_item<K, D>(ta, w, dk, cc, stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y), lane, sy, sp);
    window_exit<K, D>(a, L, wg, sy, sp);
}

// ---------------------------------------------------------------------------
// Power iteration, up to DP sweeps per launch: level j = A^j (x / ||x||)
// formed by the same streaming (no shift), the sums of squares of every
// level recorded, the last level written; the next launch scales by its norm.
// The directions are those of the normalised iteration x_{k+1} = A x_k /
// ||A x_k||, and rho_hat = ||level nlev|| / ||level nlev-1|| of the last
// launch (level 0 has norm 1).  The host bounds nlev so that the unnormalised
// levels (at most rho^j) stay far from overflow.
// Partial sums: the start vector's (power_norm_kernel) at partials[nb + i],
// launch b's at partials[2 nb + (b & 1) nb DP + i DP + j].
// ---------------------------------------------------------------------------

template <int DP>
__device__ __forceinline__ void stream_power_item(const Sten& st, const int nx, const int ny,
                                                  const double* __restrict__ in, double* __restrict__ out,
                                                  const double s, const int nlev, const StreamItem it, const int lane,
                                                  double (&sy)[DP]) {
    const int rc = 2 * lane - DP;
    const int gcol = wrap(it.xs + rc, nx);
    const bool ocol = rc >= 0 && rc < it.ws;
    const int T = it.hb + 2 * DP;
    const int ytop = it.yb - DP;
    auto row_off = [&](const int t) { return static_cast<long>(wrap(ytop + t, ny)) * nx + gcol; };
    double2 lc[DP], lq[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) lc[j] = lq[j] = double2{0.0, 0.0};
    double2 yq0 = ld_pair(in + row_off(0));
    double2 yq1 = ld_pair(in + row_off(1));
    for (int t0 = 0; t0 < T; t0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = t0 + u;
            double2 cur;
            cur.x = s * yq0.x;
            cur.y = s * yq0.y;
            yq0 = yq1;
            yq1 = ld_pair(in + row_off(t + 2 < T ? t + 2 : T - 1));
#pragma unroll
            for (int j = 1; j <= DP; ++j) {
                const double2 y = stream_complete(st, lq[j - 1], cur);
                lq[j - 1] = stream_partial(st, st.c4, lc[j - 1], cur);
                lc[j - 1] = cur;
                cur = y;
                const int r = t - j;
                if (r >= DP && r < DP + it.hb && j <= nlev && ocol) {
                    sy[j - 1] += y.x * y.x + y.y * y.y;
                    if (j == nlev) *reinterpret_cast<double2*>(out + row_off(r)) = y;
                }
            }
        }
    }
}

// Launch b makes nlev levels from `in`, scaled by the norm of the last level
// of launch b - 1 (which made prev levels) or of the start vector.
template <int DP>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void power_stream(
    PowerArgs a, const double* in, double* out, const int b, const int nlev, const int prev) {
    const int wg = static_cast<int>(blockIdx.x);
    double scale;
    if (b == 0) {
        double tot[1];
        sum_partials<1>(a.partials + a.nb, a.nb, tot);
        scale = 1.0 / sqrt(tot[0]);
    } else {
        double tot[DP];
        sum_partials<DP>(a.partials + 2L * a.nb + static_cast<long>((b - 1) & 1) * a.nb * DP, a.nb, tot);
        double last = tot[DP - 1];
#pragma unroll
        for (int j = 0; j < DP; ++j)
            if (j == prev - 1) last = tot[j];
        scale = 1.0 / sqrt(last);
    }
    const int nl = __builtin_amdgcn_readfirstlane(nlev);
    // the plain operator (no shift)
    const Sten st{a.cW, a.cE, a.cS, a.cN, a.cC, 0.0, 0.0, 0.0, 0.0};
    double sy[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) sy[j] = 0.0;
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int items = a.tiles_x * a.tiles_y, G = a.nb * kStreamWaves;
    for (int i = stream_wave(wg, a.nb); i < items; i += G)
        stream_power_item<DP>(st, a.nx, a.ny, in, out, scale, nl, stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y),
                              lane, sy);
    block_sum<DP>(sy);
    if (flat_tid() == 0) {
        double* __restrict__ Pp = a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * DP + static_cast<long>(wg) * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) Pp[j] = sy[j];
    }
}

// rho_hat = ||level nlev|| / ||level nlev-1|| of the last launch b
template <int DP>
__global__ __launch_bounds__(kBlockThreads) void power_stream_final(PowerArgs a, const int b, const int nlev) {
    double tot[DP];
    sum_partials<DP>(a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * DP, a.nb, tot);
    if (flat_tid() == 0) {
        double last = 0.0, prev = 1.0;
#pragma unroll
        for (int j = 0; j < DP; ++j) {
            if (j == nlev - 1) last = tot[j];
            if (j == nlev - 2) prev = tot[j];
        }
        a.ctl->rho = sqrt(last / prev);
    }
}

template <int K, int D>
hipError_t launch_stream_kd(const SweepArgs& a, int L, hipStream_t s) {
    hipLaunchKernelGGL((leja_stream<K, D>), dim3(a.nb), dim3(kBlockThreads), 0, s, a, L);
    return hipGetLastError();
}

}  // namespace

int stream_strips(int nx, int depth) {
    const int out_pairs = 64 - depth;   // column pairs a strip outputs
    return ((nx / 2) + out_pairs - 1) / out_pairs;
}

bool stream_has(int K, int depth) {
    return (depth == 4 && K >= 1 && K <= 4) || (depth == 6 && K >= 1 && K <= 3) || (depth == 8 && K == 1);
}

hipError_t launch_leja_stream(int K, int depth, const SweepArgs& a, int L, hipStream_t s) {
    if (!stream_has(K, depth) || a.nb < 1 || a.nx % 2 != 0 || a.nx < depth || a.ny < depth)
        return hipErrorInvalidValue;
    if (a.tiles_x != stream_strips(a.nx, depth) || a.tiles_y < 1 || a.tiles_y > a.ny) return hipErrorInvalidValue;
    switch (depth * 8 + K) {
        case 33: return launch_stream_kd<1, 4>(a, L, s);
        case 34: return launch_stream_kd<2, 4>(a, L, s);
        case 35: return launch_stream_kd<3, 4>(a, L, s);
        case 36: return launch_stream_kd<4, 4>(a, L, s);
        case 49: return launch_stream_kd<1, 6>(a, L, s);
        case 50: return launch_stream_kd<2, 6>(a, L, s);
        case 51: return launch_stream_kd<3, 6>(a, L, s);
        case 65: return launch_stream_kd<1, 8>(a, L, s);
        default: return hipErrorInvalidValue;
    }
}

int stream_resident(int K, int depth, int power) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void* k = nullptr;
    if (power) {
        k = reinterpret_cast<const void*>(power_stream<kPowerStreamDepth>);
    } else {
        switch (depth * 8 + K) {
            case 33: k = reinterpret_cast<const void*>(leja_stream<1, 4>); break;
            case 34: k = reinterpret_cast<const void*>(leja_stream<2, 4>); break;
            case 35: k = reinterpret_cast<const void*>(leja_stream<3, 4>); break;
            case 36: k = reinterpret_cast<const void*>(leja_stream<4, 4>); break;
            case 49: k = reinterpret_cast<const void*>(leja_stream<1, 6>); break;
            case 50: k = reinterpret_cast<const void*>(leja_stream<2, 6>); break;
            case 51: k = reinterpret_cast<const void*>(leja_stream<3, 6>); break;
            case 65: k = reinterpret_cast<const void*>(leja_stream<1, 8>); break;
            default: return 0;
        }
    }
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlockThreads, 0);
    return e == hipSuccess ? per_cu * cus : 0;
}

hipError_t launch_power_stream(const PowerArgs& a, const double* in, double* out, int b, int nlev, int prev,
                               hipStream_t s) {
    constexpr int DP = kPowerStreamDepth;
    if (a.nb < 1 || a.nx % 2 != 0 || a.nx < DP || a.ny < DP || nlev < 1 || nlev > DP || prev < 1 || prev > DP)
        return hipErrorInvalidValue;
    if (a.tiles_x != stream_strips(a.nx, DP) || a.tiles_y < 1 || a.tiles_y > a.ny) return hipErrorInvalidValue;
    hipLaunchKernelGGL((power_stream<DP>), dim3(a.nb), dim3(kBlockThreads), 0, s, a, in, out, b, nlev, prev);
    return hipGetLastError();
}

hipError_t launch_power_stream_final(const PowerArgs& a, int b, int nlev, hipStream_t s) {
    hipLaunchKernelGGL((power_stream_final<kPowerStreamDepth>), dim3(1), dim3(kBlockThreads), 0, s, a, b, nlev);
    return hipGetLastError();
}

}  // namespace lx
