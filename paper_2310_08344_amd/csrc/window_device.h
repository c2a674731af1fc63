// The window loop's control, shared by its two kernels: leja_block (LDS
// tiles, block.hip) and leja_stream (register streaming, stream.hip).
//
// Launch w of the plain loop advances the Newton recurrence (Sec. 2.1,
// Eq. (2)) from y_m (m = wD) through y_{m+1} .. y_{m+D}.  The stop rule
// (Sec. 2.2) for term m+j needs norms of y_{m+j} and of p_{m+j} over the
// whole grid, which exist only after the launch; a window therefore adds all
// D terms speculatively to every output still iterating and records, for
// every j, the sums of squares of y_{m+j} and of each output as it stands
// after term m+j.  The next launch applies the stop rule at m+1, .., m+D in
// turn and, if an output stopped inside the window, re-executes the window
// for the stopped outputs only, with exactly the terms they take.
#pragma once

#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"
#include "tile_device.h"

namespace lx {
namespace dev {

// v of lane l - 1 (kFromBelow: DPP wave_shr:1) or of lane l + 1 (wave_shl:1);
// the lane with no such neighbour keeps `old`.  Every lane of the wavefront
// must be active.
template <bool kFromBelow>
__device__ __forceinline__ double lane_neighbour(const double v, const double old) {
    constexpr int ctrl = kFromBelow ? 0x138 : 0x130;
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The state entering a launch from the state of the previous launch and its
// partial sums tot[(j-1)(1+K) + q], q = 0: |y_{m+j}|^2, q = 1+k: |p_k|^2
// after term m+j (j = 1..D).
//
// kFp32 (FP32 sweeps): a window forms its levels and writes y_{m+D} in FP32
// (out32) once, at the last term of the window before it, every output
// still iterating has |d| ||y|| <= fp32_switch * (rtol ||p|| + atol); from
// then on every window does.  in32: the window's y_m is stored in FP32.  A
// re-execution keeps the precision of the window it repeats.
template <int K, int D, bool kFp32 = false>
__device__ __forceinline__ SweepState block_decide(const SweepArgs& a, const LoopCtl& ctl, const SweepState& prev,
                                                   const double (&tot)[D * (1 + K)]) {
    SweepState nx = prev;
    if (prev.blk_mode == 1) {
        // the window was re-executed with its stops: the outputs that took all
        // D terms go on from y_{m+D}
        nx.blk_mode = 0;
        nx.iter = prev.iter + D;
        nx.in32 = prev.out32;
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            nx.active[k] = (prev.active[k] && prev.nt[k] == D) ? 1 : 0;
            nx.nt[k] = nx.active[k] ? D : 0;
            any = any || nx.active[k];
        }
        if (!any) nx.done = 1;
        return nx;
    }
    const int m = prev.iter;
    bool stopped = false, nonfinite = false, notconv = false;
    int nt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) nt[k] = prev.active[k] ? D : 0;
    for (int j = 1; j <= D; ++j) {
        const double ynorm = sqrt(tot[(j - 1) * (1 + K)]) * a.inv_sqrtN;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (nt[k] != D) continue;   // inactive, or stopped earlier in this window
            const double pn = sqrt(tot[(j - 1) * (1 + K) + 1 + k]) * a.inv_sqrtN;
            const double e = fabs(gptr(a.coef)[k * a.ld + m + j]) * ynorm;
            const double thr = ctl.rtol * pn + ctl.atol;
            nx.err[k] = e;
            nx.pnorm[k] = pn;
            nx.ynorm = ynorm;
            if (!isfinite(pn) || !isfinite(e)) {
                nonfinite = true;
            } else if (e <= thr) {
                nt[k] = -j;   // stopped after term m+j (also when j = D)
                nx.iters[k] = m + j;
                stopped = true;
            } else if (m + j >= ctl.max_iters) {
                nt[k] = -j;
                nx.iters[k] = m + j;
                stopped = true;
                notconv = true;
            }
        }
    }
    if (nonfinite) {
        nx.status = 4;   // LX_ENONFINITE
        nx.done = 1;
        return nx;
    }
    if (stopped) {
        // re-execute the window with the stops: nt[k] = -j for an output
        // that stopped after term m+j, D for one that goes on, 0 otherwise
        nx.blk_mode = 1;
#pragma unroll
        for (int k = 0; k < K; ++k) nx.nt[k] = nt[k];
        if (notconv) nx.status = 3;   // LX_ENOTCONV
    } else {
        nx.iter = m + D;
        nx.in32 = prev.out32;
        if (kFp32 && !prev.out32 && ctl.fp32_switch >= 0.0) {
            bool small = true;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (nt[k] == D && !(nx.err[k] <= ctl.fp32_switch * (ctl.rtol * nx.pnorm[k] + ctl.atol))) small = false;
            if (small) nx.out32 = 1;
        }
    }
    return nx;
}

// What launch L of a window loop does, decided at its entry.
template <int K>
struct WindowPlan {
    int m;                  // the window's first term index
    int win;                // window number, m / D
    bool redo;              // re-execution of a window in which an output stopped
    int nt[K];              // terms each output takes in this launch
    int jmax;               // levels this launch forms
    bool win32;             // levels formed, and y_{m+D} written, in FP32
    bool in32;              // y_m is stored in FP32
    bool copy[K];           // a re-execution copies this output unchanged (pin to pout)
    const double* pin[K];   // outputs as the window finds them
    double* pout[K];        // and where it leaves them
    const double* yin;      // y_m
    double* yout;           // y_{m+D}
};

// Entry of launch L of the window loop as workgroup `wg` of the a.nb that
// serve this grid: the decision from the previous launch's partial sums.
// Workgroup 0 records the state; when the loop has ended it publishes
// slot[2] and, if `done` is given, counts the grid as finished.  Returns
// false when this launch has nothing to do (the same in every thread).
//
// kEndCopy: in a re-execution, an output that stopped after the window's
// last term (j = D) is not recomputed: the window's own result is exact.
// An odd window wrote it to the caller's buffer already (nothing to do); an
// even window's result is copied there (WindowPlan::copy).
//
// Buffers: window w reads y_m from v (w = 0) or ybuf[(w-1) & 1] and writes
// y_{m+D} to ybuf[w & 1]; it reads the outputs from p (w even) or p2 (w odd)
// and writes them to the other; a re-execution writes stopped outputs to p,
// the caller's buffer, so every final result lands there.
template <int OP, int K, int D, bool kEndCopy = false, bool kFp32 = false>
__device__ __forceinline__ bool window_enter(const SweepArgs& a, const int L, const int wg, unsigned* done,
                                             WindowPlan<K>& w) {
    LoopCtl* __restrict__ ctl = gptr(a.ctl);
    constexpr int NV = D * (1 + K);
    __shared__ SweepState s_cur;
    const int tid = flat_tid();
    if (L == 0) {
        if (tid == 0) {
            SweepState st = ctl->slot[0];
            st.blk_mode = 0;
            st.iter = 0;
            for (int k = 0; k < kKMax; ++k) st.nt[k] = (k < K && st.active[k]) ? D : 0;
            st.n_work = 1;
            st.n_levels = D;
            st.in32 = 0;
            if (!kFp32) st.out32 = 0;
            st.n_fp32 = st.out32 ? D : 0;
            // v in, y_D out, the Burgers state, each output written
            double b = 8.0 + (st.out32 ? 4.0 : 8.0) + (OP == kOpBurgersJ ? (st.out32 ? 4.0 : 8.0) : 0.0);
            for (int k = 0; k < K; ++k) b += st.nt[k] ? 8.0 : 0.0;
            st.bytes_pp = b;
            s_cur = st;
            if (wg == 0) ctl->slot[0] = st;
        }
    } else {
        double tot[NV];
        sum_partials<NV>(gptr(a.partials) + static_cast<long>((L - 1) & 1) * a.nb * NV, a.nb, tot);
        if (tid == 0) {
            SweepState st = block_decide<K, D, kFp32>(a, *ctl, ctl->slot[(L - 1) & 1], tot);
            if (!st.done) {
                // algorithmic bytes per point: y in (and out, unless a
                // re-execution), and per output written p (in and out; the
                // first window only writes it)
                const bool rd = st.blk_mode == 1;
                st.n_work += 1;
                double b = 0.0;
                int lev = rd ? 0 : D;
                for (int k = 0; k < K; ++k) {
                    const bool end = kEndCopy && rd && st.nt[k] == -D;   // exact already: copied or kept
                    const bool w_k = rd ? (st.nt[k] < 0 && (!end || (st.iter / D) % 2 == 0)) : st.nt[k] != 0;
                    if (w_k) b += st.iter == 0 && !end ? 8.0 : 16.0;
                    if (rd && !end && -st.nt[k] > lev) lev = -st.nt[k];
                }
                // y in (and out), and u, when levels are formed
                const double yb = st.in32 ? 4.0 : 8.0, ob = st.out32 ? 4.0 : 8.0;
                if (!rd || lev > 0) b += yb + (rd ? 0.0 : ob) + (OP == kOpBurgersJ ? ob : 0.0);
                st.bytes_pp += b;
                st.n_levels += lev;
                if (!rd && st.out32) st.n_fp32 += D;
            }
            s_cur = st;
            if (wg == 0) {
                ctl->slot[L & 1] = st;
                if (st.done) {
                    publish_final(ctl, a.pub, st);   // this launch does no work
                    if (done != nullptr) atomicAdd(done, 1u);
                }
            }
        }
    }
    __syncthreads();
    if (s_cur.done) return false;
    // every field below is the same in all threads of the grid
    w.m = __builtin_amdgcn_readfirstlane(s_cur.iter);
    w.win = w.m / D;
    w.redo = __builtin_amdgcn_readfirstlane(s_cur.blk_mode) == 1;
    w.win32 = kFp32 && __builtin_amdgcn_readfirstlane(s_cur.out32) != 0;
    w.in32 = kFp32 && __builtin_amdgcn_readfirstlane(s_cur.in32) != 0;
    // terms each output takes in this launch.  A re-execution recomputes
    // only the outputs that stopped (their final buffer is p); the others,
    // and y_{m+D}, the window already wrote exactly.
    w.jmax = w.redo ? 0 : D;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = __builtin_amdgcn_readfirstlane(s_cur.nt[k]);
        const bool end = kEndCopy && w.redo && q == -D;
        w.nt[k] = (w.redo && !end) ? (q < 0 ? -q : 0) : (w.redo ? 0 : q);
        if (w.nt[k] > w.jmax) w.jmax = w.nt[k];
        // an even window wrote its outputs to p2, an odd one to p
        w.copy[k] = end && (w.win & 1) == 0;
        w.pin[k] = gptr(end ? a.p2[k] : ((w.win & 1) ? a.p2[k] : a.p[k]));
        w.pout[k] = gptr(w.redo ? a.p[k] : ((w.win & 1) ? a.p[k] : a.p2[k]));
    }
    w.yin = gptr((w.win == 0) ? a.v : static_cast<const double*>(a.ybuf[(w.win - 1) & 1]));
    w.yout = gptr(static_cast<double*>(a.ybuf[w.win & 1]));
    return true;
}

template <int K, int D>
__device__ __forceinline__ void window_exit_sums(const SweepArgs& a, int L, int wg, double (&v)[D * (1 + K)]);

// Exit of a window launch: the workgroup's sums of squares of every level
// (sy[j-1]: y_{m+j}) and of every output after each term (sp[k][j-1]), in a
// fixed order, into this workgroup's record of partials[L & 1].
template <int K, int D>
__device__ __forceinline__ void window_exit(const SweepArgs& a, const int L, const int wg, const double (&sy)[D],
                                            const double (&sp)[K][D]) {
    constexpr int NV = D * (1 + K);
    double v[NV];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        v[j * (1 + K)] = sy[j];
#pragma unroll
        for (int k = 0; k < K; ++k) v[j * (1 + K) + 1 + k] = sp[k][j];
    }
    window_exit_sums<K, D>(a, L, wg, v);
}

// The same from the packed record v[(j-1)(1+K) + q] (q = 0: y_{m+j}, 1+k:
// output k), this thread's share.
template <int K, int D>
__device__ __forceinline__ void window_exit_sums(const SweepArgs& a, const int L, const int wg,
                                                 double (&v)[D * (1 + K)]) {
    constexpr int NV = D * (1 + K);
    block_sum<NV>(v);
    if (flat_tid() == 0) {
        double* __restrict__ Pp = gptr(a.partials) + static_cast<long>(L & 1) * a.nb * NV + static_cast<long>(wg) * NV;
#pragma unroll
        for (int q = 0; q < NV; ++q) Pp[q] = v[q];
    }
}

}  // namespace dev
}  // namespace lx
