// Two Leja iterations per launch (gfx950), FP64.
//
// The single-sweep kernel moves (16 + 16K) bytes per point for every
// iteration: the basis vector in and out and each unconverged output in and
// out.  Here one launch advances the Newton recurrence (Sec. 2.1, Eq. (2))
// by two steps on LDS-resident tiles:
//
//     y_{m+1} = ((A - c)/gamma - xi_m) y_m        on the tile plus a 1-cell halo
//     y_{m+2} = ((A - c)/gamma - xi_{m+1}) y_{m+1}  on the tile
//
// so y_m is read once (with a 2-cell halo, mostly from L2) and only y_{m+2}
// is written: the same bytes as one sweep buy two iterations.
//
// The stop rule (Sec. 2.2) for term m+1 needs norms that only exist after
// the launch, so the second term is deferred: launch L (m = 2L) adds
// d_m y_m (its own input, the term deferred by launch L-1) and
// d_{m+1} y_{m+1}, and records the sums of squares of y_{m+1}, of the
// outputs after that update, of y_{m+2}, and of the outputs as they would
// be with d_{m+2} y_{m+2} added.  At the next launch every workgroup adds
// the partial sums in the same fixed order and applies the stop rule at
// terms m+1 and m+2 in turn; an output that passed at m+1 takes no further
// term, one that passes at m+2 takes only the deferred d_{m+2} y_{m+2}.
// The arithmetic on every output is the single-sweep kernel's, term by term
// in the same order, so the results and iteration counts are those of
// one-iteration launches up to the order of the norm reductions.
//
// When the rule ends the loop with a deferred term still owed, the launch
// only adds it (a "flush"), records the final state in its parity slot, and
// the following launch publishes it to slot[2]: slot[2] must not announce
// the end while workgroups of the flushing launch may still be starting.
//
// Tiles are 128 columns (64 lanes x 2) by TH rows; a workgroup is four
// wavefronts.  For a stencil of radius R (1 for the five-point operators, 2
// for third-order upwind advection) LDS holds y_m on rows -2R..TH+2R-1 and
// columns -2R..127+2R of the tile (and the Burgers state u on the same
// cells) and y_{m+1} on rows -R..TH+R-1 and columns -R..127+R.  Global
// indices wrap periodically, so cells of a tile past the grid's edge hold
// the wrapped values and the halo of the last real column is exactly the
// periodic neighbour; such cells are computed but never stored or counted.
// Requires nx even (16-byte pairs).
#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"
#include "tile_device.h"

namespace lx {
namespace {

using namespace dev;

template <int OP, int TH>
struct PairLds {
    static constexpr int R = radius<OP>();
    double ym[TH + 4 * R][pitch<R>()];      // y_m: row r at [r + 2R], column c at [c + 2R]
    double y1[TH + 2 * R][pitch<R>()];      // y_{m+1}: row r at [r + R], column c at [c + 2R]
    double u[TH + 4 * R][pitch<R>()];       // Burgers state, laid out as ym
};
template <int TH>
struct PairLds<kOpDiffAdv, TH> {
    double ym[TH + 4][pitch<1>()];
    double y1[TH + 2][pitch<1>()];
};
template <int TH>
struct PairLds<kOpDiffAdv3, TH> {
    double ym[TH + 8][pitch<2>()];
    double y1[TH + 4][pitch<2>()];
};

// y_m of one tile as this thread stages it (rows -2..TH+1 of its column
// pair, and one halo value), loaded a tile ahead of its LDS staging so that
// the loads overlap the previous tile's arithmetic
template <int TH, int R>
struct TileY {
    // the two columns of each staged row, kept as two scalar arrays (an
    // array of double2 this long is not promoted to registers)
    double x[(TH + 4 * R) / kPairWaves], y[(TH + 4 * R) / kPairWaves];
    double edge;
};

// Edge cells of y_m: 4R per staged row (LDS columns 0..2R-1 and
// 128+2R..127+4R), one per thread; thread e covers row e / 4R.
template <int TH, int R>
constexpr bool edges_fit() {
    return (TH + 4 * R) * 4 * R <= kBlockThreads;
}

template <int K, int TH, int R>
__device__ __forceinline__ TileY<TH, R> load_tile_y(const TileArgs<K>& a, const double* __restrict__ yin,
                                                    const int tile) {
    TileY<TH, R> r;
    r.edge = 0.0;
    static_assert(TH % kPairWaves == 0, "tile rows must be a multiple of the wavefronts");
    static_assert(edges_fit<TH, R>(), "one edge cell per thread");
    const int nx = a.nx, ny = a.ny;
    const int x0 = (tile % a.tiles_x) * kPairTW, y0 = (tile / a.tiles_x) * TH;
    const int tid = flat_tid(), lane = tid & 63, w = tid >> 6;
    const int gc = wrap(x0 + 2 * lane, nx);       // even: nx and x0 are even
#pragma unroll
    for (int i = 0; i < (TH + 4 * R) / kPairWaves; ++i) {
        const long g = wrap(y0 - 2 * R + w + i * kPairWaves, ny) * static_cast<long>(nx) + gc;
        const double2 t = *reinterpret_cast<const double2*>(yin + g);
        r.x[i] = t.x;
        r.y[i] = t.y;
    }
    if (tid < (TH + 4 * R) * 4 * R) {
        const int q = tid % (4 * R);
        const int ec = (q < 2 * R) ? q : kPairTW + q;
        r.edge = yin[wrap(y0 - 2 * R + tid / (4 * R), ny) * static_cast<long>(nx) + wrap(x0 + ec - 2 * R, nx)];
    }
    return r;
}

template <int OP, int K, int TH>
__device__ __forceinline__ void pair_tile(const TileArgs<K>& a, PairLds<OP, TH>& S, const double* __restrict__ yin,
                                          double* __restrict__ yout, const int m, const bool first,
                                          const int (&add0)[K], const int (&add1)[K], double& sy1, double& sy2,
                                          double (&sp1)[K], double (&sp2)[K], const int tile,
                                          TileY<TH, radius<OP>()>& ty, const int next) {
    constexpr int R = radius<OP>();
    constexpr int RW = TH / kPairWaves;           // tile rows per wavefront
    const int nx = a.nx, ny = a.ny;
    const int x0 = (tile % a.tiles_x) * kPairTW, y0 = (tile / a.tiles_x) * TH;
    const int tid = flat_tid(), lane = tid & 63, w = tid >> 6;
    const double* __restrict__ uu = a.u;
    const int j = 2 * R + 2 * lane;               // LDS column of this lane's pair
    const int gcol = x0 + 2 * lane;
    const int gc = wrap(gcol, nx);                // even: nx and x0 are even
    const double xm = a.xi[m], xm1 = a.xi[m + 1];

    // ---- y_m (and u) on rows -2R..TH+2R-1, columns -2R..127+2R; the outputs ----
    constexpr int RM = (TH + 4 * R) / kPairWaves; // staged rows of y_m per wavefront
    double uedge = 0.0;
    int er = 0, ec = 0;
    const bool has_edge = tid < (TH + 4 * R) * 4 * R;
    if (has_edge) {
        er = tid / (4 * R);
        const int q = tid % (4 * R);
        ec = (q < 2 * R) ? q : kPairTW + q;       // LDS columns 0..2R-1, 128+2R..127+4R
        if constexpr (OP == kOpBurgersJ)
            uedge = uu[wrap(y0 - 2 * R + er, ny) * static_cast<long>(nx) + wrap(x0 + ec - 2 * R, nx)];
    }
    // outputs of this thread's rows, fetched while the tile is staged
    double2 pv[K][RW];
    if (!first) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!(add0[k] | add1[k])) continue;
            const double* __restrict__ pk = a.p[k];
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const int grow = y0 + w + i * kPairWaves;
                if (gcol < nx && grow < ny)
                    pv[k][i] = ld_stream(pk + static_cast<long>(grow) * nx + gcol);
            }
        }
    }
    if constexpr (OP == kOpBurgersJ) {
#pragma unroll
        for (int i = 0; i < RM; ++i) {
            const int r = w + i * kPairWaves;
            const long g = wrap(y0 - 2 * R + r, ny) * static_cast<long>(nx) + gc;
            *reinterpret_cast<double2*>(&S.u[r][j]) = *reinterpret_cast<const double2*>(uu + g);
        }
    }
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        const int r = w + i * kPairWaves;
        double2 t;
        t.x = ty.x[i];
        t.y = ty.y[i];
        *reinterpret_cast<double2*>(&S.ym[r][j]) = t;
    }
    if (has_edge) {
        S.ym[er][ec] = ty.edge;
        if constexpr (OP == kOpBurgersJ) S.u[er][ec] = uedge;
    }
    __syncthreads();
    ty = load_tile_y<K, TH, R>(a, yin, next);   // the next tile's y_m, in flight during this one

    // ---- y_{m+1} on rows -R..TH+R-1, columns -R..127+R: LDS row r of y1
    // is centred on LDS row r + R of ym ----
#pragma unroll
    for (int i = 0; i < (TH + 2 * R + kPairWaves - 1) / kPairWaves; ++i) {
        const int r = w + i * kPairWaves;
        if (r >= TH + 2 * R) break;
        double o[2];
        if constexpr (OP == kOpDiffAdv3) {
            shifted_pair3(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], S.ym[r + 3], S.ym[r + 4], j, o);
        } else if constexpr (OP == kOpBurgersJ) {
            shifted_pair<OP>(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], S.u[r], S.u[r + 1], S.u[r + 2], j, o);
        } else {
            shifted_pair<OP>(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], nullptr, nullptr, nullptr, j, o);
        }
        double2 t;
        t.x = o[0];
        t.y = o[1];
        *reinterpret_cast<double2*>(&S.y1[r][j]) = t;
    }
    // the R columns on each side of the tile: LDS columns R..2R-1 and
    // 128+2R..127+3R
    if (tid < (TH + 2 * R) * 2 * R) {
        const int r = tid / (2 * R), q = tid % (2 * R);
        const int lc = (q < R) ? R + q : kPairTW + R + q;
        if constexpr (OP == kOpDiffAdv3) {
            S.y1[r][lc] = shifted_one3(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], S.ym[r + 3], S.ym[r + 4], lc);
        } else if constexpr (OP == kOpBurgersJ) {
            S.y1[r][lc] = shifted_one<OP>(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], S.u[r], S.u[r + 1], S.u[r + 2], lc);
        } else {
            S.y1[r][lc] = shifted_one<OP>(a.st, xm, S.ym[r], S.ym[r + 1], S.ym[r + 2], nullptr, nullptr, nullptr, lc);
        }
    }
    __syncthreads();

    // ---- y_{m+2} on the tile; outputs; sums of squares ----
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = w + i * kPairWaves;
        const int grow = y0 + r;
        double o[2];
        if constexpr (OP == kOpDiffAdv3) {
            shifted_pair3(a.st, xm1, S.y1[r], S.y1[r + 1], S.y1[r + 2], S.y1[r + 3], S.y1[r + 4], j, o);
        } else if constexpr (OP == kOpBurgersJ) {
            shifted_pair<OP>(a.st, xm1, S.y1[r], S.y1[r + 1], S.y1[r + 2], S.u[r + 1], S.u[r + 2], S.u[r + 3], j, o);
        } else {
            shifted_pair<OP>(a.st, xm1, S.y1[r], S.y1[r + 1], S.y1[r + 2], nullptr, nullptr, nullptr, j, o);
        }
        if (gcol < nx && grow < ny) {
            const long idx = static_cast<long>(grow) * nx + gcol;
            const double2 c1 = *reinterpret_cast<const double2*>(&S.y1[r + R][j]);
            const double2 c0 = *reinterpret_cast<const double2*>(&S.ym[r + 2 * R][j]);
            double2 t;
            t.x = o[0];
            t.y = o[1];
            *reinterpret_cast<double2*>(yout + idx) = t;
            sy1 += c1.x * c1.x + c1.y * c1.y;
            sy2 += o[0] * o[0] + o[1] * o[1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!(add0[k] | add1[k])) continue;
                const double dm = a.coef[k * a.ld + m], dm1 = a.coef[k * a.ld + m + 1];
                const double dm2 = a.coef[k * a.ld + m + 2];
                double2 p;
                if (first) {
                    // p_0 = d_0 y_0; y_0 = v is the centre
                    p.x = dm * c0.x;
                    p.y = dm * c0.y;
                } else {
                    p = pv[k][i];
                    if (add0[k]) {
                        p.x = fma(dm, c0.x, p.x);
                        p.y = fma(dm, c0.y, p.y);
                    }
                }
                if (add1[k]) {
                    p.x = fma(dm1, c1.x, p.x);
                    p.y = fma(dm1, c1.y, p.y);
                }
                st_stream(a.p[k] + idx, p);
                sp1[k] += p.x * p.x + p.y * p.y;
                const double qx = fma(dm2, o[0], p.x), qy = fma(dm2, o[1], p.y);
                sp2[k] += qx * qx + qy * qy;
            }
        }
    }
    __syncthreads();   // the next tile overwrites LDS
}

// One launch L of the two-iteration loop, as workgroup `wg` of the `a.nb`
// that serve this grid: the stop decisions at terms 2L-1 and 2L from the
// previous launch's partial sums, then the flush or the two sweeps.
// Workgroup 0 records the state; when the loop has ended it also publishes
// slot[2] and, if `done` is given, counts the grid as finished.  `banded`
// selects the XCD-banded tile order (whole-device grids).
template <int OP, int K, int TH>
__device__ __forceinline__ void pair_launch(const SweepArgs& a, const int L, const int wg, const bool banded,
                                            PairLds<OP, TH>& S, unsigned* done) {
    LoopCtl* __restrict__ ctl = gptr(a.ctl);
    constexpr int NV = 2 * (1 + K);
    __shared__ int s_mode;   // 0: both terms, 1: deferred term only, 2: nothing
    __shared__ int s_add0[K], s_add1[K];
    const int tid = flat_tid();
    const int m = 2 * L;
    if (L == 0) {
        if (tid == 0) {
            s_mode = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                s_add0[k] = 1;
                s_add1[k] = ctl->slot[0].active[k];
            }
        }
    } else {
        double tot[NV];
        sum_partials<NV>(gptr(a.partials) + static_cast<long>((L - 1) & 1) * a.nb * NV, a.nb, tot);
        if (tid == 0) {
            const SweepState prev = ctl->slot[(L - 1) & 1];
            const bool pub = wg == 0;
            if (prev.done) {
                // the previous launch flushed the last deferred term
                s_mode = 2;
                if (pub) {
                    publish_final(ctl, a.pub, prev);
                    if (done != nullptr) atomicAdd(done, 1u);
                }
            } else {
                double t1[1 + K], t2[1 + K];
                t1[0] = tot[0];
                t2[0] = tot[1 + K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    t1[1 + k] = tot[1 + k];
                    t2[1 + k] = tot[2 + K + k];
                }
                const SweepState s1 = decide<K, false>(a, *ctl, prev, m - 1, t1);
                if (s1.done) {
                    s_mode = 2;
                    if (pub) {
                        ctl->slot[L & 1] = s1;
                        publish_final(ctl, a.pub, s1);
                        if (done != nullptr) atomicAdd(done, 1u);
                    }
                } else {
                    const SweepState s2 = decide<K, false>(a, *ctl, s1, m, t2);
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        s_add0[k] = s1.active[k];
                        s_add1[k] = s2.done ? 0 : s2.active[k];
                    }
                    s_mode = s2.done ? 1 : 0;
                    if (pub) ctl->slot[L & 1] = s2;
                }
            }
        }
    }
    __syncthreads();
    const int mode = s_mode;
    if (mode == 2) return;
    int add0[K], add1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        add0[k] = s_add0[k];
        add1[k] = s_add1[k];
    }
    const double* __restrict__ yin = gptr((L == 0) ? a.v : static_cast<const double*>(a.ybuf[(L - 1) & 1]));

    if (mode == 1) {
        // p_k += d_m y_m for the outputs that passed the stop rule at term m
        const long n2 = static_cast<long>(a.nx) * a.ny / 2;
        for (long i = static_cast<long>(wg) * kBlockThreads + tid; i < n2; i += static_cast<long>(a.nb) * kBlockThreads) {
            const double2 y = reinterpret_cast<const double2*>(yin)[i];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!add0[k]) continue;
                const double dm = gptr(a.coef)[k * a.ld + m];
                double2 p = reinterpret_cast<const double2*>(gptr(a.p[k]))[i];
                p.x = fma(dm, y.x, p.x);
                p.y = fma(dm, y.y, p.y);
                reinterpret_cast<double2*>(gptr(a.p[k]))[i] = p;
            }
        }
        return;
    }

    double* __restrict__ yout = gptr(static_cast<double*>(a.ybuf[L & 1]));
    double sy1 = 0.0, sy2 = 0.0, sp1[K], sp2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sp1[k] = 0.0;
        sp2[k] = 0.0;
    }
    const int T = a.tiles_x * a.tiles_y;
    const TileArgs<K> ta = tile_args<OP, K>(a);
    // this workgroup's tiles: first, first + step, ... < end (an XCD's band
    // for whole-device grids, a contiguous run for a batch instance)
    int first, step, end;
    if (banded && a.nb >= 8 && (a.nb & 7) == 0) {
        const int x = wg & 7, nbx = a.nb >> 3;
        first = static_cast<int>((static_cast<long>(x) * T) >> 3) + (wg >> 3);
        step = nbx;
        end = static_cast<int>((static_cast<long>(x + 1) * T) >> 3);
    } else if (banded) {
        first = wg;
        step = a.nb;
        end = T;
    } else {
        first = static_cast<int>((static_cast<long>(wg) * T) / a.nb);
        step = 1;
        end = static_cast<int>((static_cast<long>(wg + 1) * T) / a.nb);
    }
    TileY<TH, radius<OP>()> ty;
    if (first < end) ty = load_tile_y<K, TH, radius<OP>()>(ta, yin, first);
    for (int t = first; t < end; t += step) {
        // after the last tile, reload it (from L2) rather than branch: the
        // registers then stay registers
        const int next = (t + step < end) ? t + step : t;
        pair_tile<OP, K, TH>(ta, S, yin, yout, m, L == 0, add0, add1, sy1, sy2, sp1, sp2, t, ty, next);
    }
    double v[NV];
    v[0] = sy1;
    v[1 + K] = sy2;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[1 + k] = sp1[k];
        v[2 + K + k] = sp2[k];
    }
    block_sum<NV>(v);
    if (tid == 0) {
        double* __restrict__ P = gptr(a.partials) + static_cast<long>(L & 1) * a.nb * NV + static_cast<long>(wg) * NV;
#pragma unroll
        for (int q = 0; q < NV; ++q) P[q] = v[q];
    }
}

template <int OP, int K, int TH>
__global__ __launch_bounds__(kBlockThreads) void leja_pair(SweepArgs a, const int L) {
    if (loop_ended(gptr(a.ctl))) return;
    __shared__ PairLds<OP, TH> S;
    pair_launch<OP, K, TH>(a, L, static_cast<int>(blockIdx.x), true, S, nullptr);
}

// Batched: every workgroup serves the instance block_inst[blockIdx.x], one
// output per instance; LDS is sized by the launch for the largest tile
// layout in the batch.
template <int TH>
__global__ __launch_bounds__(kBlockThreads) void batch_pair_kernel(const BatchInst* insts, LoopCtl* ctls,
                                                                   const int* block_inst, double* partials,
                                                                   const double* coef, const int ld,
                                                                   const double* xi, unsigned* done, const int L) {
    extern __shared__ double lds_dyn[];
    // the instance's arguments live in LDS: a per-lane copy would be indexed
    // dynamically (the basis parity) and spill to scratch
    __shared__ SweepArgs a;
    const int i = block_inst[blockIdx.x];
    const BatchInst& I = insts[i];
    LoopCtl* __restrict__ ctl = ctls + i;
    if (loop_ended(ctl)) return;
    if (flat_tid() == 0) {
        a = SweepArgs{};
        a.nx = I.nx;
        a.ny = I.ny;
        a.tiles_x = I.tiles_x;
        a.tiles_y = I.tiles_y;
        a.nb = I.nb;
        a.ld = ld;
        if (I.kind == kOpDiffAdv) {
            a.aE = I.st[0];
            a.aW = I.st[1];
            a.aN = I.st[2];
            a.aS = I.st[3];
            a.aC = I.st[4];
        } else {
            a.kx = I.st[0];
            a.ky = I.st[1];
            a.gx = I.st[2];
            a.gy = I.st[3];
            a.kC = I.st[4];
        }
        a.inv_sqrtN = 1.0 / sqrt(static_cast<double>(I.nx) * I.ny);
        a.v = I.v;
        a.ybuf[0] = I.y[0];
        a.ybuf[1] = I.y[1];
        a.u = I.u;
        a.p[0] = I.out;
        a.coef = coef + static_cast<long>(i) * ld;
        a.xi = xi;
        a.partials = partials + I.part_off;
        a.ctl = ctl;
    }
    __syncthreads();
    const int wg = static_cast<int>(blockIdx.x) - I.wg_begin;
    if (I.kind == kOpDiffAdv) {
        pair_launch<kOpDiffAdv, 1, TH>(a, L, wg, false, *reinterpret_cast<PairLds<kOpDiffAdv, TH>*>(lds_dyn), done);
    } else {
        pair_launch<kOpBurgersJ, 1, TH>(a, L, wg, false, *reinterpret_cast<PairLds<kOpBurgersJ, TH>*>(lds_dyn), done);
    }
}

template <int OP, int K>
hipError_t launch_pair_th(int th, const SweepArgs& a, int L, hipStream_t s) {
    const dim3 block(64, kPairWaves), grid(a.nb);
    switch (th) {
        case 8: hipLaunchKernelGGL((leja_pair<OP, K, 8>), grid, block, 0, s, a, L); break;
        case 16: hipLaunchKernelGGL((leja_pair<OP, K, 16>), grid, block, 0, s, a, L); break;
        case 32:
            if constexpr (edges_fit<32, radius<OP>()>()) {
                hipLaunchKernelGGL((leja_pair<OP, K, 32>), grid, block, 0, s, a, L);
            } else {
                return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int OP>
hipError_t launch_pair_k(int K, int th, const SweepArgs& a, int L, hipStream_t s) {
    switch (K) {
        case 1: return launch_pair_th<OP, 1>(th, a, L, s);
        case 2: return launch_pair_th<OP, 2>(th, a, L, s);
        case 3: return launch_pair_th<OP, 3>(th, a, L, s);
        case 4: return launch_pair_th<OP, 4>(th, a, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch_pair(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks, bool burgers,
                             int th, double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                             int L, hipStream_t s) {
    if (nblocks < 1) return hipErrorInvalidValue;
    const dim3 block(64, kPairWaves), grid(nblocks);
    switch (th) {
        case 8: {
            const size_t lds = burgers ? sizeof(PairLds<kOpBurgersJ, 8>) : sizeof(PairLds<kOpDiffAdv, 8>);
            hipLaunchKernelGGL(batch_pair_kernel<8>, grid, block, lds, s, insts, ctls, block_inst, partials, coef, ld, xi,
                               done, L);
            break;
        }
        case 16: {
            const size_t lds = burgers ? sizeof(PairLds<kOpBurgersJ, 16>) : sizeof(PairLds<kOpDiffAdv, 16>);
            hipLaunchKernelGGL(batch_pair_kernel<16>, grid, block, lds, s, insts, ctls, block_inst, partials, coef, ld,
                               xi, done, L);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_leja_pair(int op, int K, int th, const SweepArgs& a, int L, hipStream_t s) {
    if (a.nb < 1 || a.nx % 2 != 0 || a.nx < 2 || a.ny < 2) return hipErrorInvalidValue;
    if (a.tiles_x != (a.nx + kPairTW - 1) / kPairTW || a.tiles_y != (a.ny + th - 1) / th)
        return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_pair_k<kOpDiffAdv>(K, th, a, L, s);
    if (op == kOpBurgersJ) return launch_pair_k<kOpBurgersJ>(K, th, a, L, s);
    if (op == kOpDiffAdv3) {
        if (a.nx < 4 || a.ny < 4) return hipErrorInvalidValue;   // wrap() reaches back 2R = 4 cells
        return launch_pair_k<kOpDiffAdv3>(K, th, a, L, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lx
