// D Leja iterations per launch (D = 3, 4 or 6) on LDS-resident tiles (gfx950),
// FP64, with speculative windows.
//
// Launch w of the plain loop advances the Newton recurrence (Sec. 2.1,
// Eq. (2)) from y_m (m = wD) through y_{m+1} .. y_{m+D} on a tile staged
// once with a D-cell halo (D R cells for a stencil of radius R), so the
// basis vector is read and written once and every output once per D
// iterations.  The stop rule (Sec. 2.2) for term m+j needs norms of
// y_{m+j} and of p_{m+j} over the whole grid, which exist only after the
// launch; the window therefore adds all D terms speculatively to every
// output still iterating and records, for every j, the sums of squares of
// y_{m+j} and of each output as it stands after term m+j.  The outputs of a
// window go to a second buffer, so its inputs survive it.
//
// The next launch adds the partial sums (the same fixed order in every
// workgroup) and applies the stop rule at m+1, .., m+D in turn.  If no output
// stopped inside the window, the speculation was exact and the loop goes on
// from y_{m+D}.  If some did, the launch re-executes the window from the same
// inputs with the terms each output really takes (up to its stopping term),
// writing stopped outputs to their final buffer; y_{m+D} and the outputs
// that go on come out bitwise as before (explicit-FMA stencils, the same
// terms in the same order).  Every output therefore takes exactly the terms
// of the one-iteration loop, in the same order, and the iteration counts are
// those of one-iteration launches up to the order of the norm reductions.
//
// Buffers: window w reads y_m from v (w = 0) or ybuf[(w-1) & 1] and writes
// y_{m+D} to ybuf[w & 1]; it reads the outputs from p (w even) or p2 (w odd)
// and writes them to the other; a re-execution writes stopped outputs to p,
// the caller's buffer, so every final result lands there.
//
// Tiles are 128 columns by TH rows, four wavefronts; LDS holds two levels
// (ping-pong) of ROWS = TH + 2H rows and 128 + 2H (rounded up to even)
// columns, H = D R: level j
// is valid on the tile plus an (D - j) R halo, and level D is formed in
// registers on the tile only.
#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"
#include "tile_device.h"
#include "window_device.h"

namespace lx {
namespace {

using namespace dev;

template <int OP, int TH, int D>
struct BlockLds {
    static constexpr int R = radius<OP>();
    static constexpr int H = D * R;              // halo of level 0
    static constexpr int CO = (H + 1) & ~1;      // column offset: even, so column pairs are 16-byte aligned
    static constexpr int ROWS = TH + 2 * H;
    static constexpr int P = kPairTW + 2 * CO;   // row pitch in doubles
    double a[ROWS][P];                           // levels 0, 2, ...: LDS row r = tile row r - H,
    double b[ROWS][P];                           // levels 1, 3, ...: LDS column c = tile column c - CO
    static constexpr bool kHasU = false;
    __device__ const double (*uu() const)[P] { return nullptr; }
};
// the Burgers Jacobian also reads the state u on the level-0 cells
template <int TH, int D>
struct BlockLds<kOpBurgersJ, TH, D> {
    static constexpr int R = 1, H = D, CO = (H + 1) & ~1, ROWS = TH + 2 * H, P = kPairTW + 2 * CO;
    double a[ROWS][P];
    double b[ROWS][P];
    double u[ROWS][P];
    static constexpr bool kHasU = true;
    __device__ const double (*uu() const)[P] { return u; }
};

// y_m of one tile as this thread stages it, loaded a tile ahead
template <int TH, int D, int R>
struct BlockY {
    static constexpr int H = D * R, ROWS = TH + 2 * H;
    static constexpr int RM = (ROWS + kPairWaves - 1) / kPairWaves;   // rows per wavefront
    static constexpr int E = ROWS * 2 * H;                             // edge cells
    static constexpr int EQ = (E + kBlockThreads - 1) / kBlockThreads; // edge cells per thread
    double x[RM], y[RM];
    double edge[EQ];
};

template <int K, int TH, int D, int R>
__device__ __forceinline__ BlockY<TH, D, R> load_block_y(const TileArgs<K>& a, const double* __restrict__ yin,
                                                         const int tile) {
    using Y = BlockY<TH, D, R>;
    constexpr int H = Y::H;
    Y r;
    const int nx = a.nx, ny = a.ny;
    const int x0 = (tile % a.tiles_x) * kPairTW, y0 = (tile / a.tiles_x) * TH;
    const int tid = flat_tid(), lane = tid & 63, w = tid >> 6;
    const int gc = wrap(x0 + 2 * lane, nx);       // even: nx and x0 are even
#pragma unroll
    for (int i = 0; i < Y::RM; ++i) {
        const int row = w + i * kPairWaves;
        r.x[i] = 0.0;
        r.y[i] = 0.0;
        if (row < Y::ROWS) {
            const long g = wrap(y0 - H + row, ny) * static_cast<long>(nx) + gc;
            const double2 t = *reinterpret_cast<const double2*>(yin + g);
            r.x[i] = t.x;
            r.y[i] = t.y;
        }
    }
#pragma unroll
    for (int q = 0; q < Y::EQ; ++q) {
        const int e = tid + q * kBlockThreads;
        r.edge[q] = 0.0;
        if (e < Y::E) {
            // tile column -H .. -1 (qq < H) or 128 .. 127+H
            const int row = e / (2 * H), qq = e % (2 * H);
            const int tc = (qq < H) ? qq - H : kPairTW + (qq - H);
            r.edge[q] = yin[wrap(y0 - H + row, ny) * static_cast<long>(nx) + wrap(x0 + tc, nx)];
        }
    }
    return r;
}

// Row `ce` around the column pair j, j+1 of this lane, where the 64 lanes of
// the wavefront hold the pairs of 128 consecutive columns (j = j_0 + 2 lane):
// c = {ce[j], ce[j+1]}, l = {ce[j-2], ce[j-1]}, r = {ce[j+2], ce[j+3]}.  The
// side columns come from the neighbouring lanes' pairs; only lanes 0 and 63
// read theirs, the halo beyond the wavefront's columns, from LDS.
__device__ __forceinline__ void row_pair(const double* ce, const int j, double2& c, double2& l, double2& r) {
    const int lane = flat_tid() & 63;
    c = *reinterpret_cast<const double2*>(ce + j);
    double2 e = double2{0.0, 0.0};
    if (lane == 0 || lane == 63) e = *reinterpret_cast<const double2*>(ce + (lane == 0 ? j - 2 : j + 2));
    l.x = lane_neighbour<true>(c.x, e.x);
    l.y = lane_neighbour<true>(c.y, e.y);
    r.x = lane_neighbour<false>(c.x, e.x);
    r.y = lane_neighbour<false>(c.y, e.y);
}

// the shifted operator at the column pair j, j+1 of LDS row r of `src`
// (u: the Burgers state laid out as src, else NULL).  The five-point
// diffusion-advection operator takes a wavefront's row of 128 columns at once
// (row_pair): every lane of the wavefront calls this with j = j_0 + 2 lane;
// the stencil and its operand order are those of shifted_pair.  (The
// radius-2 operator reads its four side columns from LDS: exchanging them
// between lanes measured slower.)
template <int OP, int P>
__device__ __forceinline__ void level_pair(const Sten& st, const double shift, const double (*src)[P], const int r,
                                           const int j, double (&o)[2], const double (*u)[P] = nullptr) {
    if constexpr (radius<OP>() == 2) {
        shifted_pair3(st, shift, src[r - 2], src[r - 1], src[r], src[r + 1], src[r + 2], j, o);
    } else if constexpr (OP == kOpBurgersJ) {
        shifted_pair<OP>(st, shift, src[r - 1], src[r], src[r + 1], u[r - 1], u[r], u[r + 1], j, o);
    } else {
        double2 c, l, rr;
        row_pair(src[r], j, c, l, rr);
        const double2 s = *reinterpret_cast<const double2*>(src[r - 1] + j);
        const double2 n = *reinterpret_cast<const double2*>(src[r + 1] + j);
        o[0] = shifted_at<OP>(st, shift, l.y, c.y, s.x, n.x, c.x, 0, 0, 0, 0);
        o[1] = shifted_at<OP>(st, shift, c.x, rr.x, s.y, n.y, c.y, 0, 0, 0, 0);
    }
}

template <int OP, int P>
__device__ __forceinline__ double level_one(const Sten& st, const double shift, const double (*src)[P], const int r,
                                            const int j, const double (*u)[P] = nullptr) {
    if constexpr (radius<OP>() == 2) {
        return shifted_one3(st, shift, src[r - 2], src[r - 1], src[r], src[r + 1], src[r + 2], j);
    } else if constexpr (OP == kOpBurgersJ) {
        return shifted_one<OP>(st, shift, src[r - 1], src[r], src[r + 1], u[r - 1], u[r], u[r + 1], j);
    } else {
        return shifted_one<OP>(st, shift, src[r - 1], src[r], src[r + 1], nullptr, nullptr, nullptr, j);
    }
}

template <int OP, int K, int TH, int D>
__device__ __forceinline__ void block_tile(const TileArgs<K>& a, BlockLds<OP, TH, D>& S,
                                           const double* __restrict__ yin, double* __restrict__ yout,
                                           const double* const (&pin)[K], double* const (&pout)[K], const int m,
                                           const bool first, const int (&nt)[K], const int jmax,
                                           const bool store_y, double (&sy)[D],
                                           double (&sp)[K][D], const int tile, BlockY<TH, D, radius<OP>()>& ty,
                                           const int next) {
    using L = BlockLds<OP, TH, D>;
    using Y = BlockY<TH, D, radius<OP>()>;
    constexpr int R = L::R, H = L::H, CO = L::CO, ROWS = L::ROWS, P = L::P;
    constexpr int RW = TH / kPairWaves;           // tile rows per wavefront
    const int nx = a.nx, ny = a.ny;
    const int x0 = (tile % a.tiles_x) * kPairTW, y0 = (tile / a.tiles_x) * TH;
    const int tid = flat_tid(), lane = tid & 63, w = tid >> 6;
    const int j0 = CO + 2 * lane;                 // LDS column of this lane's pair
    const int gcol = x0 + 2 * lane;

    // ---- the outputs of this thread's rows, fetched while the tile is staged ----
    double2 pv[K][RW];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int i = 0; i < RW; ++i) pv[k][i] = double2{0.0, 0.0};
        if (first || nt[k] == 0) continue;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int grow = y0 + w + i * kPairWaves;
            if (gcol < nx && grow < ny) pv[k][i] = ld_stream(pin[k] + static_cast<long>(grow) * nx + gcol);
        }
    }
    // ---- the Burgers state on the level-0 cells (the same every launch: L2) ----
    if constexpr (L::kHasU) {
        const double* __restrict__ uu = a.u;
        const int gc = wrap(gcol, nx);
        for (int r = w; r < ROWS; r += kPairWaves)
            *reinterpret_cast<double2*>(&S.u[r][j0]) =
                *reinterpret_cast<const double2*>(uu + wrap(y0 - H + r, ny) * static_cast<long>(nx) + gc);
        for (int e = tid; e < Y::E; e += kBlockThreads) {
            const int row = e / (2 * H), qq = e % (2 * H);
            const int tc = (qq < H) ? qq - H : kPairTW + (qq - H);
            S.u[row][CO + tc] = uu[wrap(y0 - H + row, ny) * static_cast<long>(nx) + wrap(x0 + tc, nx)];
        }
    }
    // ---- level 0: y_m on rows -H..TH+H-1, columns -H..127+H ----
#pragma unroll
    for (int i = 0; i < Y::RM; ++i) {
        const int r = w + i * kPairWaves;
        if (r < ROWS) {
            double2 t;
            t.x = ty.x[i];
            t.y = ty.y[i];
            *reinterpret_cast<double2*>(&S.a[r][j0]) = t;
        }
    }
#pragma unroll
    for (int q = 0; q < Y::EQ; ++q) {
        const int e = tid + q * kBlockThreads;
        if (e < Y::E) {
            const int row = e / (2 * H), qq = e % (2 * H);
            const int tc = (qq < H) ? qq - H : kPairTW + (qq - H);
            S.a[row][CO + tc] = ty.edge[q];
        }
    }
    __syncthreads();
    ty = load_block_y<K, TH, D, R>(a, yin, next);   // the next tile's y_m, in flight during this one
    if (first) {
        // p_0 = d_0 y_0
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const double2 c0 = *reinterpret_cast<const double2*>(&S.a[H + w + i * kPairWaves][j0]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double d0 = gptr(a.coef)[k * a.ld];
                pv[k][i].x = d0 * c0.x;
                pv[k][i].y = d0 * c0.y;
            }
        }
    }

    // ---- levels 1 .. D-1 in LDS, each followed by the terms it gives
    // (up to level jmax, the same in every thread) ----
#pragma unroll
    for (int j = 1; j < D; ++j) {
        if (j > jmax) break;
        const double (*src)[P] = ((j - 1) & 1) ? S.b : S.a;
        double (*dst)[P] = (j & 1) ? S.b : S.a;
        const double shift = gptr(a.xi)[m + j - 1];
        const int r_lo = j * R, r_hi = ROWS - j * R;    // level j on LDS rows [r_lo, r_hi)
#pragma unroll
        for (int i = 0; i < (ROWS + kPairWaves - 1) / kPairWaves; ++i) {
            const int r = r_lo + w + i * kPairWaves;
            if (r < r_hi) {
                double o[2];
                level_pair<OP, P>(a.st, shift, src, r, j0, o, S.uu());
                double2 t;
                t.x = o[0];
                t.y = o[1];
                *reinterpret_cast<double2*>(&dst[r][j0]) = t;
            }
        }
        // the (D - j) R columns on each side of the tile
        const int side = H - j * R;
        const int ne = (r_hi - r_lo) * 2 * side;
        for (int e = tid; e < ne; e += kBlockThreads) {
            const int r = r_lo + e / (2 * side), qq = e % (2 * side);
            const int tc = (qq < side) ? qq - side : kPairTW + (qq - side);
            dst[r][CO + tc] = level_one<OP, P>(a.st, shift, src, r, CO + tc, S.uu());
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int grow = y0 + w + i * kPairWaves;
            if (gcol < nx && grow < ny) {
                const double2 y = *reinterpret_cast<const double2*>(&dst[H + w + i * kPairWaves][j0]);
                sy[j - 1] += y.x * y.x + y.y * y.y;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (nt[k] < j) continue;
                    const double dj = gptr(a.coef)[k * a.ld + m + j];
                    pv[k][i].x = fma(dj, y.x, pv[k][i].x);
                    pv[k][i].y = fma(dj, y.y, pv[k][i].y);
                    sp[k][j - 1] += pv[k][i].x * pv[k][i].x + pv[k][i].y * pv[k][i].y;
                }
            }
        }
    }

    // ---- level D on the tile: y_{m+D} and the last term ----
    if (jmax >= D) {
        const double (*src)[P] = ((D - 1) & 1) ? S.b : S.a;
        const double shift = gptr(a.xi)[m + D - 1];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int r = H + w + i * kPairWaves;
            const int grow = y0 + w + i * kPairWaves;
            double o[2];
            level_pair<OP, P>(a.st, shift, src, r, j0, o, S.uu());
            if (gcol < nx && grow < ny) {
                const long idx = static_cast<long>(grow) * nx + gcol;
                if (store_y) {
                    double2 t;
                    t.x = o[0];
                    t.y = o[1];
                    *reinterpret_cast<double2*>(yout + idx) = t;
                }
                sy[D - 1] += o[0] * o[0] + o[1] * o[1];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (nt[k] < D) continue;
                    const double dD = gptr(a.coef)[k * a.ld + m + D];
                    pv[k][i].x = fma(dD, o[0], pv[k][i].x);
                    pv[k][i].y = fma(dD, o[1], pv[k][i].y);
                    sp[k][D - 1] += pv[k][i].x * pv[k][i].x + pv[k][i].y * pv[k][i].y;
                }
            }
        }
    }
    // ---- the outputs ----
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int grow = y0 + w + i * kPairWaves;
        if (gcol < nx && grow < ny) {
            const long idx = static_cast<long>(grow) * nx + gcol;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (nt[k] > 0) st_stream(pout[k] + idx, pv[k][i]);
        }
    }
    __syncthreads();   // the next tile overwrites LDS
}

// One launch L of the window loop as workgroup `wg` of the a.nb that serve
// this grid: the decision, then the window, its re-execution or nothing.
// Workgroup 0 records the state; when the loop has ended it publishes
// slot[2] and, if `done` is given, counts the grid as finished.  `banded`
// selects the XCD-banded tile order (whole-device grids), else each
// workgroup takes a contiguous run of tiles (a batch instance).
template <int OP, int K, int TH, int D>
__device__ __forceinline__ void block_launch(const SweepArgs& a, const int L, const int wg, const bool banded,
                                             BlockLds<OP, TH, D>& S, unsigned* done) {
    WindowPlan<K> w;
    if (!window_enter<OP, K, D>(a, L, wg, done, w)) return;
    double sy[D], sp[K][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sy[j] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sp[k][j] = 0.0;
    }
    const int T = a.tiles_x * a.tiles_y;
    const TileArgs<K> ta = tile_args<OP, K>(a);
    // this workgroup's tiles: a band of its XCD, as in the two-iteration
    // kernel, or a contiguous run (batch instances)
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
    BlockY<TH, D, radius<OP>()> ty;
    if (first < end) ty = load_block_y<K, TH, D, radius<OP>()>(ta, w.yin, first);
    for (int t = first; t < end; t += step) {
        const int next = (t + step < end) ? t + step : t;
        block_tile<OP, K, TH, D>(ta, S, w.yin, w.yout, w.pin, w.pout, w.m, w.win == 0, w.nt, w.jmax, !w.redo, sy,
                                 sp, t, ty, next);
    }
    window_exit<K, D>(a, L, wg, sy, sp);
}

template <int OP, int K, int TH, int D>
__global__ __launch_bounds__(kBlockThreads) void leja_block(SweepArgs a, const int L) {
    if (loop_ended(gptr(a.ctl))) return;
    __shared__ BlockLds<OP, TH, D> S;
    block_launch<OP, K, TH, D>(a, L, static_cast<int>(blockIdx.x), true, S, nullptr);
}

// Batched windows: every workgroup serves the instance block_inst[blockIdx.x],
// one output per instance; LDS is sized by the launch for the largest
// layout in the batch (the Burgers one when the batch holds one).
template <int TH, int D>
__global__ __launch_bounds__(kBlockThreads) void batch_block_kernel(const BatchInst* insts, LoopCtl* ctls,
                                                                    const int* block_inst, double* partials,
                                                                    const double* coef, const int ld,
                                                                    const double* xi, unsigned* done, const int L) {
    extern __shared__ double lds_dyn[];
    // the instance's arguments live in LDS (a per-lane copy would be indexed
    // dynamically and spill to scratch)
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
        a.p2[0] = I.out2;
        a.coef = coef + static_cast<long>(i) * ld;
        a.xi = xi;
        a.partials = partials + I.part_off;
        a.ctl = ctl;
    }
    __syncthreads();
    const int wg = static_cast<int>(blockIdx.x) - I.wg_begin;
    if (I.kind == kOpDiffAdv) {
        block_launch<kOpDiffAdv, 1, TH, D>(a, L, wg, false, *reinterpret_cast<BlockLds<kOpDiffAdv, TH, D>*>(lds_dyn),
                                           done);
    } else {
        block_launch<kOpBurgersJ, 1, TH, D>(a, L, wg, false,
                                            *reinterpret_cast<BlockLds<kOpBurgersJ, TH, D>*>(lds_dyn), done);
    }
}

// ---------------------------------------------------------------------------
// power iteration, D sweeps per launch: level j = A^j (x / ||x||) on the tile
// (levels 1..nlev-1 in LDS, the last in registers), the sums of squares of
// every level recorded; the next launch scales by the last level's norm.
// The directions are those of the normalised iteration x_{k+1} = A x_k /
// ||A x_k||; rho_hat = ||level nlev|| / ||level nlev-1|| (level 0 has norm
// 1).  Unnormalised levels grow like rho_hat^j, far from overflow for any
// stencil of practical size.
// ---------------------------------------------------------------------------

template <int OP, int TH, int D>
__device__ __forceinline__ void power_block_tile(const TileArgs<1>& ta, const Sten& st, BlockLds<OP, TH, D>& S,
                                                 const double* __restrict__ in, double* __restrict__ out,
                                                 const double s, const int nlev, double (&sy)[D], const int tile,
                                                 BlockY<TH, D, radius<OP>()>& ty, const int next) {
    using L = BlockLds<OP, TH, D>;
    using Y = BlockY<TH, D, radius<OP>()>;
    constexpr int R = L::R, H = L::H, CO = L::CO, ROWS = L::ROWS, P = L::P;
    constexpr int RW = TH / kPairWaves;
    const int nx = ta.nx, ny = ta.ny;
    const int x0 = (tile % ta.tiles_x) * kPairTW, y0 = (tile / ta.tiles_x) * TH;
    const int tid = flat_tid(), lane = tid & 63, w = tid >> 6;
    const int j0 = CO + 2 * lane;
    const int gcol = x0 + 2 * lane;
    // the Burgers state on the level-0 cells (the same every launch: L2)
    if constexpr (L::kHasU) {
        const double* __restrict__ uu = ta.u;
        const int gc = wrap(gcol, nx);
        for (int r = w; r < ROWS; r += kPairWaves)
            *reinterpret_cast<double2*>(&S.u[r][j0]) =
                *reinterpret_cast<const double2*>(uu + wrap(y0 - H + r, ny) * static_cast<long>(nx) + gc);
        for (int e = tid; e < Y::E; e += kBlockThreads) {
            const int row = e / (2 * H), qq = e % (2 * H);
            const int tc = (qq < H) ? qq - H : kPairTW + (qq - H);
            S.u[row][CO + tc] = uu[wrap(y0 - H + row, ny) * static_cast<long>(nx) + wrap(x0 + tc, nx)];
        }
    }
#pragma unroll
    for (int i = 0; i < Y::RM; ++i) {
        const int r = w + i * kPairWaves;
        if (r < ROWS) {
            double2 t;
            t.x = s * ty.x[i];
            t.y = s * ty.y[i];
            *reinterpret_cast<double2*>(&S.a[r][j0]) = t;
        }
    }
#pragma unroll
    for (int q = 0; q < Y::EQ; ++q) {
        const int e = tid + q * kBlockThreads;
        if (e < Y::E) {
            const int row = e / (2 * H), qq = e % (2 * H);
            const int tc = (qq < H) ? qq - H : kPairTW + (qq - H);
            S.a[row][CO + tc] = s * ty.edge[q];
        }
    }
    __syncthreads();
    ty = load_block_y<1, TH, D, R>(ta, in, next);
#pragma unroll
    for (int j = 1; j < D; ++j) {
        if (j >= nlev) break;
        const double (*src)[P] = ((j - 1) & 1) ? S.b : S.a;
        double (*dst)[P] = (j & 1) ? S.b : S.a;
        const int r_lo = j * R, r_hi = ROWS - j * R;
#pragma unroll
        for (int i = 0; i < (ROWS + kPairWaves - 1) / kPairWaves; ++i) {
            const int r = r_lo + w + i * kPairWaves;
            if (r < r_hi) {
                double o[2];
                level_pair<OP, P>(st, 0.0, src, r, j0, o, S.uu());
                double2 t;
                t.x = o[0];
                t.y = o[1];
                *reinterpret_cast<double2*>(&dst[r][j0]) = t;
            }
        }
        const int side = H - j * R;
        const int ne = (r_hi - r_lo) * 2 * side;
        for (int e = tid; e < ne; e += kBlockThreads) {
            const int r = r_lo + e / (2 * side), qq = e % (2 * side);
            const int tc = (qq < side) ? qq - side : kPairTW + (qq - side);
            dst[r][CO + tc] = level_one<OP, P>(st, 0.0, src, r, CO + tc, S.uu());
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int grow = y0 + w + i * kPairWaves;
            if (gcol < nx && grow < ny) {
                const double2 y = *reinterpret_cast<const double2*>(&dst[H + w + i * kPairWaves][j0]);
                sy[j - 1] += y.x * y.x + y.y * y.y;
            }
        }
    }
    {
        const double (*src)[P] = ((nlev - 1) & 1) ? S.b : S.a;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int grow = y0 + w + i * kPairWaves;
            double o[2];
            level_pair<OP, P>(st, 0.0, src, H + w + i * kPairWaves, j0, o, S.uu());
            if (gcol < nx && grow < ny) {
                double2 t;
                t.x = o[0];
                t.y = o[1];
                *reinterpret_cast<double2*>(out + static_cast<long>(grow) * nx + gcol) = t;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (j == nlev - 1) sy[j] += o[0] * o[0] + o[1] * o[1];
            }
        }
    }
    __syncthreads();
}

// Partial sums: the start vector's (power_norm_kernel) at partials[nb + i];
// launch b's at partials[2 nb + (b & 1) nb D + i D + j].
template <int OP, int TH, int D>
__global__ __launch_bounds__(kBlockThreads) void power_block(PowerArgs a, const double* in, double* out, const int b,
                                                             const int nlev) {
    constexpr int R = radius<OP>();
    __shared__ BlockLds<OP, TH, D> S;
    const int tid = flat_tid();
    const int wg = static_cast<int>(blockIdx.x);
    double scale;
    if (b == 0) {
        double tot[1];
        sum_partials<1>(a.partials + a.nb, a.nb, tot);
        scale = 1.0 / sqrt(tot[0]);
    } else {
        double tot[D];
        sum_partials<D>(a.partials + 2L * a.nb + static_cast<long>((b - 1) & 1) * a.nb * D, a.nb, tot);
        scale = 1.0 / sqrt(tot[D - 1]);   // every launch but the last makes D levels
    }
    TileArgs<1> ta{};
    ta.nx = a.nx;
    ta.ny = a.ny;
    ta.tiles_x = a.tiles_x;
    ta.u = a.u;
    // the plain operator (no shift): the Burgers centre as the one-sweep
    // power iteration forms it
    const Sten st = OP == kOpBurgersJ ? Sten{a.kx, a.ky, a.gx, a.gy, -2.0 * a.kx - 2.0 * a.ky, 0.0, 0.0, 0.0, 0.0}
                                      : Sten{a.cW, a.cE, a.cS, a.cN, a.cC, a.cW2, a.cE2, a.cS2, a.cN2};
    double sy[D];
#pragma unroll
    for (int j = 0; j < D; ++j) sy[j] = 0.0;
    const int T = a.tiles_x * a.tiles_y;
    int first, step, end;
    if (a.nb >= 8 && (a.nb & 7) == 0) {
        const int x = wg & 7, nbx = a.nb >> 3;
        first = static_cast<int>((static_cast<long>(x) * T) >> 3) + (wg >> 3);
        step = nbx;
        end = static_cast<int>((static_cast<long>(x + 1) * T) >> 3);
    } else {
        first = wg;
        step = a.nb;
        end = T;
    }
    BlockY<TH, D, R> ty;
    if (first < end) ty = load_block_y<1, TH, D, R>(ta, in, first);
    for (int t = first; t < end; t += step) {
        const int next = (t + step < end) ? t + step : t;
        power_block_tile<OP, TH, D>(ta, st, S, in, out, scale, nlev, sy, t, ty, next);
    }
    block_sum<D>(sy);
    if (tid == 0) {
        double* __restrict__ Pp = a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * D + static_cast<long>(wg) * D;
#pragma unroll
        for (int j = 0; j < D; ++j) Pp[j] = sy[j];
    }
}

// rho_hat = ||level nlev|| / ||level nlev-1|| of the last launch b
template <int D>
__global__ __launch_bounds__(kBlockThreads) void power_block_final(PowerArgs a, const int b, const int nlev) {
    double tot[D];
    sum_partials<D>(a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * D, a.nb, tot);
    if (flat_tid() == 0) {
        double last = 0.0, prev = 1.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j == nlev - 1) last = tot[j];
            if (j == nlev - 2) prev = tot[j];
        }
        a.ctl->rho = sqrt(last / prev);
    }
}

// gfx950 gives a workgroup up to 160 KB of LDS; keep two workgroups per CU
template <int OP, int TH, int D>
constexpr bool block_fits() {
    return sizeof(BlockLds<OP, TH, D>) <= 78 * 1024;
}

template <int OP, int K, int D>
hipError_t launch_block_th(int th, const SweepArgs& a, int L, hipStream_t s) {
    const dim3 block(64, kPairWaves), grid(a.nb);
    switch (th) {
        case 8: hipLaunchKernelGGL((leja_block<OP, K, 8, D>), grid, block, 0, s, a, L); break;
        case 16:
            if constexpr (block_fits<OP, 16, D>()) {
                hipLaunchKernelGGL((leja_block<OP, K, 16, D>), grid, block, 0, s, a, L);
            } else {
                return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int OP, int D>
hipError_t launch_block_k(int K, int th, const SweepArgs& a, int L, hipStream_t s) {
    switch (K) {
        case 1: return launch_block_th<OP, 1, D>(th, a, L, s);
        case 2: return launch_block_th<OP, 2, D>(th, a, L, s);
        case 3: return launch_block_th<OP, 3, D>(th, a, L, s);
        case 4: return launch_block_th<OP, 4, D>(th, a, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int power_block_rows(int op) { return op == kOpDiffAdv ? 16 : 8; }

int power_block_resident(int op) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void* k = op == kOpDiffAdv3   ? reinterpret_cast<const void*>(power_block<kOpDiffAdv3, 8, kPowerBlockDepth>)
                    : op == kOpBurgersJ ? reinterpret_cast<const void*>(power_block<kOpBurgersJ, 8, kPowerBlockDepth>)
                                        : reinterpret_cast<const void*>(power_block<kOpDiffAdv, 16, kPowerBlockDepth>);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlockThreads, 0);
    return e == hipSuccess ? per_cu * cus : 0;
}

hipError_t launch_power_block(int op, const PowerArgs& a, const double* in, double* out, int b, int nlev,
                              hipStream_t s) {
    constexpr int D = kPowerBlockDepth;
    if (op != kOpDiffAdv && op != kOpDiffAdv3 && op != kOpBurgersJ) return hipErrorInvalidValue;
    if (op == kOpBurgersJ && a.u == nullptr) return hipErrorInvalidValue;
    const int TH = power_block_rows(op), H = D * (op == kOpDiffAdv3 ? 2 : 1);
    if (a.nb < 1 || a.nx % 2 != 0 || a.nx < H || a.ny < H || nlev < 1 || nlev > D) return hipErrorInvalidValue;
    if (a.tiles_x != (a.nx + kPairTW - 1) / kPairTW || a.tiles_y != (a.ny + TH - 1) / TH) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) {
        hipLaunchKernelGGL((power_block<kOpDiffAdv, 16, D>), dim3(a.nb), dim3(64, kPairWaves), 0, s, a, in, out, b,
                           nlev);
    } else if (op == kOpDiffAdv3) {
        hipLaunchKernelGGL((power_block<kOpDiffAdv3, 8, D>), dim3(a.nb), dim3(64, kPairWaves), 0, s, a, in, out, b,
                           nlev);
    } else {
        hipLaunchKernelGGL((power_block<kOpBurgersJ, 8, D>), dim3(a.nb), dim3(64, kPairWaves), 0, s, a, in, out, b,
                           nlev);
    }
    return hipGetLastError();
}

hipError_t launch_power_block_final(const PowerArgs& a, int b, int nlev, hipStream_t s) {
    hipLaunchKernelGGL((power_block_final<kPowerBlockDepth>), dim3(1), dim3(kBlockThreads), 0, s, a, b, nlev);
    return hipGetLastError();
}

hipError_t launch_batch_block(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks, bool burgers,
                              int th, double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                              int L, hipStream_t s) {
    constexpr int D = kBatchBlockDepth;
    if (nblocks < 1) return hipErrorInvalidValue;
    const dim3 block(64, kPairWaves), grid(nblocks);
    switch (th) {
        case 8: {
            const size_t lds = burgers ? sizeof(BlockLds<kOpBurgersJ, 8, D>) : sizeof(BlockLds<kOpDiffAdv, 8, D>);
            hipLaunchKernelGGL((batch_block_kernel<8, D>), grid, block, lds, s, insts, ctls, block_inst, partials, coef,
                               ld, xi, done, L);
            break;
        }
        case 16: {
            if (burgers) return hipErrorInvalidValue;   // 78 KB: batches with Burgers take 8-row tiles
            const size_t lds = sizeof(BlockLds<kOpDiffAdv, 16, D>);
            hipLaunchKernelGGL((batch_block_kernel<16, D>), grid, block, lds, s, insts, ctls, block_inst, partials,
                               coef, ld, xi, done, L);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_leja_block(int op, int K, int th, int depth, const SweepArgs& a, int L, hipStream_t s) {
    if (a.nb < 1 || a.nx % 2 != 0 || a.nx < 2 || a.ny < 2) return hipErrorInvalidValue;
    if (a.tiles_x != (a.nx + kPairTW - 1) / kPairTW || a.tiles_y != (a.ny + th - 1) / th)
        return hipErrorInvalidValue;
    const int H = depth * (op == kOpDiffAdv3 ? 2 : 1);
    if (a.nx < H || a.ny < H) return hipErrorInvalidValue;   // halo reach
    if (op == kOpDiffAdv) {
        if (depth == 3) return launch_block_k<kOpDiffAdv, 3>(K, th, a, L, s);
        if (depth == 4) return launch_block_k<kOpDiffAdv, 4>(K, th, a, L, s);
        if (depth == 6) return launch_block_k<kOpDiffAdv, 6>(K, th, a, L, s);
    } else if (op == kOpBurgersJ) {
        if (a.u == nullptr) return hipErrorInvalidValue;
        if (depth == 3) return launch_block_k<kOpBurgersJ, 3>(K, th, a, L, s);
        if (depth == 4) return launch_block_k<kOpBurgersJ, 4>(K, th, a, L, s);
    } else {
        if (depth == 3) return launch_block_k<kOpDiffAdv3, 3>(K, th, a, L, s);
        if (depth == 4) return launch_block_k<kOpDiffAdv3, 4>(K, th, a, L, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lx
