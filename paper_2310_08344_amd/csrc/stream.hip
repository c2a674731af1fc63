// Windows of D Leja iterations per launch by register streaming (gfx950),
// for the five-point diffusion-advection operator and the Burgers Jacobian,
// FP64 or FP32 levels; and power iteration with many sweeps per launch in
// the same way.
//
// The window semantics are those of leja_block (window_device.h): every
// output takes the one-iteration loop's terms in the same order, and the
// stop rule (Sec. 2.2) is applied at every term m+1 .. m+D from the sums of
// squares the window records.  Only the way the levels are formed differs.
//
// Every wavefront works alone on an item: a strip of 128 columns (64 lanes,
// a column pair each) and a band of rows, marched from top to bottom with no
// barrier.  Its 128 columns are the item's output columns and D columns on
// each side; level j (the basis vector y_{m+j}) is valid on the strip minus
// j columns on each side, so after D levels the output columns remain.
// Rows are staged from D above the band to D below it.  At step t the
// wavefront takes row t of y_m (level 0) and then forms level j at row t - j
// for j = 1..D from the two rows of level j-1 it kept in registers and the
// row of level j-1 it just formed (the Newton recurrence of Sec. 2.1,
// Eq. (2)).  The side neighbours of a column pair come from the neighbouring
// lanes (DPP wavefront shifts).  Nothing is formed twice along y (the
// LDS-tile kernel forms up to 1.7 points per output point at D = 6 on 8-row
// tiles); along x the strip's side columns are formed by two wavefronts
// (128 columns per at most 128 - 2D outputs).
//
// The outputs: for the diffusion-advection operator (ring windows, below)
// every level also goes into a small ring in LDS and the outputs of row
// t - D take all their terms at step t; otherwise (the Burgers Jacobian) an
// output row enters the registers when level 0 reaches it, takes term j
// when level j does, and leaves after its last term, D + 1 rows of every
// output in flight.  Rings of depth 7 or 8 (28 KB or 35 KB per wavefront)
// leave room in LDS for one wavefront per SIMD: those windows have a kernel
// of their own, allowed the registers of a single wavefront.
//
// Each wavefront's items are a contiguous run of bands of one XCD, so the
// side columns a neighbouring strip also loads come from that XCD's L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lx_device.h"
#include "sweep_device.h"
#include "tile_device.h"
#include "window_device.h"

namespace lx {
namespace {

using namespace dev;

constexpr int kStreamWaves = kBlockThreads / 64;   // wavefronts per workgroup, each on its own items

// Columns [xs, xs + ws) and rows [yb, yb + hb) of item i: items are numbered
// band-major over sx strips and by bands; strip edges are multiples of
// strip_unit columns.
struct StreamItem {
    int xs, ws, yb, hb;
};

// Strip edges fall on 128-byte lines (16 FP64 columns) where that costs at
// most four of a strip's 128 - 2 depth output columns, else on column pairs.
// An output row segment that ends inside a line shares that line with the
// neighbouring strip, and the nontemporal output loads then fetch it twice
// (the shared line does not stay in L2 between the two wavefronts' loads).
__host__ __device__ constexpr int strip_unit(const int nx, const int depth) {
    return (nx % 16 == 0 && (128 - 2 * depth) % 16 <= 4) ? 16 : 2;
}

__device__ __forceinline__ StreamItem stream_geom(const int i, const int nx, const int ny, const int sx,
                                                  const int by, const int unit) {
    const int b = i / sx, s = i - b * sx;
    const long units = nx / unit;
    StreamItem it;
    it.xs = unit * static_cast<int>((s * units) / sx);
    it.ws = unit * static_cast<int>(((s + 1) * units) / sx) - it.xs;
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

template <typename T>
using P2 = typename Pair<T>::type;

// v of lane l - 1 (kFromBelow: DPP wave_shr:1) or of lane l + 1
// (wave_shl:1), one DPP move per 32 bits; lane 0 (lane 63) has no such
// neighbour and reads 0.  Those lanes hold the outermost halo columns of a
// strip, which no output column depends on (level j is valid j columns in
// from the strip's edges).  Every lane of the wavefront must be active.
template <bool kFromBelow>
__device__ __forceinline__ int lane_move(const int v) {
    return __builtin_amdgcn_mov_dpp(v, kFromBelow ? 0x138 : 0x130, 0xf, 0xf, true);
}

template <bool kFromBelow, typename T>
__device__ __forceinline__ T nbr(const T v) {
    if constexpr (sizeof(T) == sizeof(double)) {
        const int lo = lane_move<kFromBelow>(__double2loint(v));
        const int hi = lane_move<kFromBelow>(__double2hiint(v));
        return __hiloint2double(hi, lo);
    } else {
        return __int_as_float(lane_move<kFromBelow>(__float_as_int(v)));
    }
}

// The stencil's coefficients in the arithmetic of the levels: c0..c3 and
// the unshifted centre c4 (Sten's order; the shifted centres are per level).
template <typename T>
struct StenT {
    T c0, c1, c2, c3;
};

template <typename T>
__device__ __forceinline__ StenT<T> sten_as(const Sten& s) {
    return StenT<T>{static_cast<T>(s.c0), static_cast<T>(s.c1), static_cast<T>(s.c2), static_cast<T>(s.c3)};
}

// The five-point diffusion-advection operator of shifted_at, split in two
// so that a level keeps only two rows in registers: stream_partial takes
// this lane's column pair of row C (the side columns from the neighbouring
// lanes) and the row S before it, and forms everything but the last term;
// stream_complete adds the term of the row N after it.  The operand order is
// stencil_da's:
//   fma(cN, N, fma(cS, S, fma(cE, E, fma(cW, W, cC C)))),
// so every kernel forms the same bits (in either precision).  All 64 lanes
// must be active.
template <typename T>
__device__ __forceinline__ P2<T> stream_partial(const StenT<T>& st, const T cc, const P2<T> S, const P2<T> C) {
#pragma clang fp contract(off)
    const T w = nbr<true>(C.y);    // column j - 1: lane - 1's second column
    const T e = nbr<false>(C.x);   // column j + 2: lane + 1's first column
    P2<T> o;
    o.x = fma(st.c2, S.x, fma(st.c1, C.y, fma(st.c0, w, cc * C.x)));
    o.y = fma(st.c2, S.y, fma(st.c1, e, fma(st.c0, C.x, cc * C.y)));
    // formed here, not where the next step uses it: the neighbour values
    // (convergent cross-lane moves, which stay put) would otherwise be held
    // in registers across the step
    asm volatile("" : "+v"(o.x), "+v"(o.y));
    return o;
}

template <typename T>
__device__ __forceinline__ P2<T> stream_complete(const StenT<T>& st, const P2<T> q, const P2<T> N) {
    P2<T> o;
    o.x = fma(st.c3, N.x, q.x);
    o.y = fma(st.c3, N.y, q.y);
    return o;
}

// The Burgers Jacobian J(u) (stencil_bu, the same operands in the same
// order as every other kernel) on this lane's column pair of row C, with the
// rows S before and N after it and the state u on those rows; the side
// columns of C and of u on C come from the neighbouring lanes.  All 64 lanes
// must be active.
template <typename T>
__device__ __forceinline__ P2<T> stream_burgers(const StenT<T>& k, const T kc, const P2<T> S, const P2<T> C,
                                                const P2<T> N, const P2<T> uS, const P2<T> uC, const P2<T> uN) {
    const T w = nbr<true>(C.y), e = nbr<false>(C.x);
    const T uw = nbr<true>(uC.y), ue = nbr<false>(uC.x);
    P2<T> o;
    o.x = stencil_bu<T>(k.c0, k.c1, k.c2, k.c3, kc, w, C.y, S.x, N.x, C.x, uw, uC.y, uS.x, uN.x);
    o.y = stencil_bu<T>(k.c0, k.c1, k.c2, k.c3, kc, C.x, e, S.y, N.y, C.y, uC.x, ue, uS.y, uN.y);
    return o;
}

__device__ __forceinline__ double2 ld_pair(const double* p) { return *reinterpret_cast<const double2*>(p); }

// A column pair of a stored vector: from FP32 storage (f32, widened
// exactly) or FP64.
__device__ __forceinline__ double2 ld_level64(const void* base, const long off, const bool f32) {
    if (f32) {
        const float2 f = *reinterpret_cast<const float2*>(static_cast<const float*>(base) + off);
        return double2{static_cast<double>(f.x), static_cast<double>(f.y)};
    }
    return ld_pair(static_cast<const double*>(base) + off);
}

// The Burgers state's column pair in T: the FP64 state or its FP32 copy.
template <typename T>
__device__ __forceinline__ P2<T> ld_state(const void* base, const long off) {
    if constexpr (sizeof(T) == sizeof(double)) return ld_pair(static_cast<const double*>(base) + off);
    else return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + off);
}

template <typename T>
__device__ __forceinline__ double2 as_d2(const P2<T> v) {
    return double2{static_cast<double>(v.x), static_cast<double>(v.y)};
}

template <typename T>
__device__ __forceinline__ P2<T> as_t2(const double2 v) {
    return P2<T>{static_cast<T>(v.x), static_cast<T>(v.y)};
}

template <typename T>
__device__ __forceinline__ P2<T> as_t2(const float2 v) {
    return P2<T>{static_cast<T>(v.x), static_cast<T>(v.y)};
}

// One item of a window launch (see the file comment), the levels in T (FP64,
// or FP32 for FP32 sweeps: the basis vectors and the stencil arithmetic;
// the outputs, the terms d_{m+j} y_{m+j} and the sums of squares stay FP64).
// dk[k][j] = d_{m+j} of output k, cc[j-1] the centre coefficient of level j.
//
// Diffusion-advection: entering step t, lc[j] holds level j at row t-j-1
// and lq[j] level j+1 at row t-j-1 without its last term; the step
// completes level j+1 there with level j at row t-j, which it has just
// formed.  Burgers: lq[j] holds level j at row t-j-2 and lc[j] at row t-j-1,
// and the step forms level j+1 at row t-j-1 whole once level j at row t-j
// exists; ur[i] holds u at row t-i (D + 2 rows: level j needs u on rows
// t-j-1 .. t-j+1).  Every step forms all D levels: before step 2j, level j is
// formed on rows whose inputs are not all staged yet, but such rows only
// feed rows of higher levels that are equally invalid, and no output row is
// among them (outputs start at row D).  A re-execution forms the levels up
// to the last term an output that stopped inside the window takes, and
// takes only those terms; outputs that stopped after the window's last term
// are copied (or kept) instead of recomputed (window_enter).  pr[k][i] holds
// output k at row t-1-i; slots of rows outside the band take no terms and
// are not stored.  Steps run in pairs, which the roles of lc and lq repeat
// with, so that they stay in place; an odd count adds one step past the
// staged rows that stores nothing.
template <int OP, int K, int D, typename T>
__device__ __forceinline__ void stream_window_item(const TileArgs<K>& ta, const WindowPlan<K>& w,
                                                   const void* __restrict__ ustate, const double (&dk)[K][D + 1],
                                                   const double (&cc)[D], const StreamItem it, const int lane,
                                                   double (&sy)[D], double (&sp)[K][D]) {
    constexpr bool BU = OP == kOpBurgersJ;
    const int nx = ta.nx, ny = ta.ny;
    const int rc = 2 * lane - D;                 // strip column of this lane's pair
    const int gcol = wrap(it.xs + rc, nx);       // even: xs, D and nx are
    const bool ocol = rc >= 0 && rc < it.ws;
    const double mcol = ocol ? 1.0 : 0.0;        // weight of this lane in the sums
    const int T_ = it.hb + 2 * D;                // rows staged: the band and D above and below
    const int ytop = it.yb - D;
    const bool first = w.win == 0, store_y = !w.redo && w.yout != nullptr;
    const bool levels = w.jmax > 0;              // a re-execution that only copies reads no y
    const bool in32 = sizeof(T) == sizeof(float) && w.in32;   // y_m stored in FP32 (FP32 levels only)
    const void* __restrict__ yin = w.yin;
    const StenT<T> st = sten_as<T>(ta.st);
    auto row_off = [&](const int t) { return static_cast<long>(wrap(ytop + t, ny)) * nx + gcol; };

    P2<T> lc[D], lq[D];
    P2<T> ur[BU ? D + 2 : 1];
    double2 pr[K][D];
#pragma unroll
    for (int j = 0; j < D; ++j) lc[j] = lq[j] = P2<T>{0, 0};
#pragma unroll
    for (int i = 0; i < (BU ? D + 2 : 1); ++i) ur[i] = P2<T>{0, 0};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) pr[k][i] = double2{0.0, 0.0};
    // Loads run ahead of their use, as far as registers allow without spills
    // at two wavefronts per SIMD: level 0 three rows ahead with at most eight
    // output rows in flight (K D) and the five-point operator in FP64, else
    // two; each output row fetched one step before it enters (used two steps
    // after its load is issued) with at most twelve, except K = 2, D = 6,
    // else in the step it enters.  The Burgers state u (in T: the FP32 copy
    // for FP32 levels) rides with level 0.
    constexpr int YQ = (K * D <= 8 && !BU && sizeof(T) == sizeof(double)) ? 3 : 2;
    constexpr bool PFP = K * D <= 12 && !(K == 2 && D == 6);
    // level 0 is held as stored, exactly (its FP64 value gives p_0 = d_0 y_0)
    double2 yq0{0.0, 0.0}, yq1{0.0, 0.0}, yq2{0.0, 0.0};
    P2<T> uq0{0, 0}, uq1{0, 0};
    if (levels) {
        yq0 = ld_level64(yin, row_off(0), in32);
        yq1 = ld_level64(yin, row_off(1), in32);
        if (YQ == 3) yq2 = ld_level64(yin, row_off(2), in32);
        if constexpr (BU) {
            uq0 = ld_state<T>(ustate, row_off(0));
            uq1 = ld_state<T>(ustate, row_off(1));
        }
    }
    double2 pf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pf[k] = double2{0.0, 0.0};   // row 0 is no output row (D >= 1)

    // steps in pairs, unrolled (the roles of lc and lq repeat with them and
    // stay in place) except at depth 6, where the unrolled pair needs more
    // registers than two wavefronts per SIMD leave
    constexpr int kPair = D == 6 ? 1 : 2;
    for (int t0 = 0; t0 < T_; t0 += 2) {
#pragma unroll kPair
        for (int u = 0; u < 2; ++u) {
            const int t = t0 + u;
            const double2 cur64 = yq0;
            P2<T> cur = as_t2<T>(cur64);
            yq0 = yq1;
            if (YQ == 3) {
                yq1 = yq2;
                if (levels) yq2 = ld_level64(yin, row_off(t + 3 < T_ ? t + 3 : T_ - 1), in32);
            } else if (levels) {
                yq1 = ld_level64(yin, row_off(t + 2 < T_ ? t + 2 : T_ - 1), in32);
            }
            if constexpr (BU) {
#pragma unroll
                for (int i = D + 1; i > 0; --i) ur[i] = ur[i - 1];
                ur[0] = uq0;   // u at row t
                uq0 = uq1;
                if (levels) uq1 = ld_state<T>(ustate, row_off(t + 2 < T_ ? t + 2 : T_ - 1));
            }
            // an output row enters when level 0 reaches it; the next one is
            // fetched now
            double2 pn[K];
            const bool orow0 = t >= D && t < D + it.hb;
            const bool orow1 = t + 1 >= D && t + 1 < D + it.hb;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                // the first window starts from p_0 = d_0 y_0 (also when it is
                // re-executed); a copy reads the window's own result
                const bool fk = first && !w.copy[k];
                const bool rd = !fk && (w.nt[k] > 0 || w.copy[k]) && ocol;
                if constexpr (PFP) {
                    pn[k] = pf[k];
                    if (fk) {
                        pn[k].x = dk[k][0] * cur64.x;
                        pn[k].y = dk[k][0] * cur64.y;
                    }
                    if (orow1 && rd) pf[k] = ld_stream(w.pin[k] + row_off(t + 1));
                } else {
                    pn[k].x = dk[k][0] * cur64.x;
                    pn[k].y = dk[k][0] * cur64.y;
                    if (orow0 && rd) pn[k] = ld_stream(w.pin[k] + row_off(t));
                }
            }
#pragma unroll
            for (int j = 1; j <= D; ++j) {
                // a re-execution forms only the levels its terms need
                if (j > w.jmax) continue;
                // cur: level j-1 at row t-j+1; y: level j at row t-j
                P2<T> y;
                const T ccj = static_cast<T>(cc[j - 1]);
                if constexpr (BU) {
                    y = stream_burgers<T>(st, ccj, lq[j - 1], lc[j - 1], cur, ur[j + 1], ur[j], ur[j - 1]);
                    lq[j - 1] = lc[j - 1];
                    lc[j - 1] = cur;
                } else {
                    y = stream_complete<T>(st, lq[j - 1], cur);
                    lq[j - 1] = stream_partial<T>(st, ccj, lc[j - 1], cur);
                    lc[j - 1] = cur;
                }
                cur = y;
                const double2 y64 = as_d2<T>(y);
                // masks as factors, not selects: a select of a product
                // becomes a branch, which splits the step into blocks
                const int r = t - j;
                const bool take = r >= D && r < D + it.hb && j <= w.jmax;
                const double m = take ? mcol : 0.0;
                sy[j - 1] = fma(m, y64.x * y64.x + y64.y * y64.y, sy[j - 1]);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool tk = take && w.nt[k] >= j;
                    const double d = tk ? dk[k][j] : 0.0;   // no term: p + 0 y
                    double2& p = pr[k][j - 1];
                    p.x = fma(d, y64.x, p.x);
                    p.y = fma(d, y64.y, p.y);
                    sp[k][j - 1] = fma(tk ? mcol : 0.0, p.x * p.x + p.y * p.y, sp[k][j - 1]);
                }
            }
            // row t-D is complete: y_{m+D} and every output that took terms
            // (an output that stopped after term j < D has not changed since)
            if (t >= 2 * D && t < T_ && ocol) {
                const long o = row_off(t - D);
                if (store_y) *reinterpret_cast<P2<T>*>(reinterpret_cast<T*>(w.yout) + o) = cur;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (w.nt[k] > 0 || w.copy[k]) st_stream(w.pout[k] + o, pr[k][D - 1]);
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

// A re-execution that forms no level only copies outputs that stopped after
// the last term of an even window from that window's buffer to the
// caller's: each lane copies its column pair of the item's band, eight rows
// in flight per output.
template <int K>
__device__ __forceinline__ void stream_copy_item(const WindowPlan<K>& w, const StreamItem it, const int lane,
                                                 const int nx) {
    const int c = 2 * lane;
    if (c >= it.ws) return;
    const long col = it.xs + c;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!w.copy[k]) continue;
        for (int r0 = 0; r0 < it.hb; r0 += 8) {
            double2 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (r0 + i < it.hb) v[i] = ld_stream(w.pin[k] + static_cast<long>(it.yb + r0 + i) * nx + col);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (r0 + i < it.hb) st_stream(w.pout[k] + static_cast<long>(it.yb + r0 + i) * nx + col, v[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Ring windows (the five-point diffusion-advection operator, D <= 6).
//
// The same levels as stream_window_item, formed the same way, but the
// outputs are completed D steps later: level j of row t - j, formed at step
// t, also goes into a ring in LDS, and at step t the outputs of row t - D
// take their terms 1 .. D in order from the rings (level D is the one just
// formed).  An output row is then one row of registers for one step, not
// D rows for D steps, so three outputs at depth six fit one wavefront, and
// every row loaded for a later step sits in a register of its own that is
// read once and then loaded again: nothing loaded is moved, so no step waits
// for the loads it has just issued.  Loads and stores go through buffer
// resources and every step issues the same ones; rows and lanes that must
// not be touched get offsets past the end of the buffer (the hardware reads
// zeros and writes nothing), so the wait for a load counts exactly the
// memory operations issued after it.  Results, sums of squares and the
// order of every operation are those of stream_window_item.
//
// Ring of level j (1 <= j < D): Ring<D>::size(j) >= D - j slots of one row
// (64 lanes x a column pair), a power of two: row r in slot r mod size.  At
// step t the slot of row t - D is read before row t - j is written (the
// only rows alive are t - D .. t - j - 1).  The step loop is unrolled by a
// multiple of every ring size, so every slot is a fixed LDS offset.
// ---------------------------------------------------------------------------

template <int D>
struct Ring {
    static constexpr int size(const int j) {
        int s = 1;
        while (s < D - j) s *= 2;
        return s;
    }
    static constexpr int base(const int j) {
        int b = 0;
        for (int i = 1; i < j; ++i) b += size(i);
        return b;
    }
    static constexpr int slots = base(D);              // rows per wavefront
    static constexpr int unroll = size(1) < 4 ? 4 : size(1);
    static constexpr int ahead_y = 4;                   // level 0 loaded this many steps ahead
    static constexpr int ahead_p = 2;                   // output rows loaded this many steps ahead
    static_assert(unroll % ahead_y == 0 && unroll % ahead_p == 0 && unroll % 2 == 0, "ring unroll");
};

template <int OP, int D>
constexpr bool kRingWindows = OP == kOpDiffAdv && D >= 3 && D <= 8;

// ring windows whose rings leave room for one wavefront per SIMD
template <int OP, int D>
constexpr bool kDeepRing = kRingWindows<OP, D> && D >= 7;

// Buffer resources (raw, byte offsets).  An offset at or past the size
// reads zeros and writes nothing; kFar is past every buffer a ring window
// takes (vectors of at most kFar bytes), and a lane offset plus a row
// offset, each at most kFar, stays below 2^32.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr unsigned kFar = 1u << 30;
constexpr int kRsrcWord3 = 0x00020000;   // gfx9 resource word 3: 32-bit elements, no swizzle
constexpr int kNontemporal = 2;

__device__ __forceinline__ Rsrc make_rsrc(const void* p, const unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), kRsrcWord3);
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <typename S, int kAux = 0>
__device__ __forceinline__ S buf_ld(const Rsrc r, const unsigned voff, const unsigned soff) {
    if constexpr (sizeof(S) == 16) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(voff), static_cast<int>(soff), kAux);
        S o;
        o.x = __hiloint2double(static_cast<int>(v.y), static_cast<int>(v.x));
        o.y = __hiloint2double(static_cast<int>(v.w), static_cast<int>(v.z));
        return o;
    } else {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff), static_cast<int>(soff), kAux);
        S o;
        o.x = __uint_as_float(v.x);
        o.y = __uint_as_float(v.y);
        return o;
    }
}

template <typename S, int kAux = 0>
__device__ __forceinline__ void buf_st(const S d, const Rsrc r, const unsigned voff) {
    if constexpr (sizeof(S) == 16) {
        u32x4 v;
        v.x = static_cast<unsigned>(__double2loint(d.x));
        v.y = static_cast<unsigned>(__double2hiint(d.x));
        v.z = static_cast<unsigned>(__double2loint(d.y));
        v.w = static_cast<unsigned>(__double2hiint(d.y));
        __builtin_amdgcn_raw_buffer_store_b128(v, r, static_cast<int>(voff), 0, kAux);
    } else {
        u32x2 v;
        v.x = __float_as_uint(d.x);
        v.y = __float_as_uint(d.y);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, static_cast<int>(voff), 0, kAux);
    }
}

// What a ring window launch does, the same for every item: the buffers
// (sized 0 where nothing is read or written), the coefficients with the
// terms each output takes (dk[k][j] = d_{m+j}, 0 past its last term) and
// the levels' centres.
template <int K, int D>
struct RingWin {
    int nx, ny;
    Sten st;
    double cc[D];
    double dk[K][D + 1];  // [k][0] unused
    Rsrc yin, yout;      // y_m (level 0), y_{m+D}
    Rsrc base[K];        // the rows each output starts from: p, or y_m in the first window
    Rsrc pout[K];
    double s0[K];        // first window: d_m for an output that starts from d_m y_m, else 1
};

// One item of a ring window.  kFirst: the first window (outputs that start
// from d_m y_m); kIn32: y_m stored in FP32 (FP32 levels only); J: the
// levels formed, D in a window, fewer in a re-execution whose outputs take
// no term past J (it writes no y); kShared: every output starts from the
// rows of base[0] (a first window without copies: y_m), loaded once per
// step.  ring: this wavefront's Ring<D>::slots rows, lane-major.
template <int K, int D, typename T, bool kFirst, bool kIn32, int J = D, bool kShared = false>
__device__ __forceinline__ void ring_window_item(const RingWin<K, D>& rw, const StreamItem it, const int lane,
                                                 P2<T>* __restrict__ ring, double (&sy)[D], double (&sp)[K][D]) {
    using R = Ring<D>;
    using Y0 = typename std::conditional<kIn32, float2, double2>::type;   // level 0 as stored
    constexpr int Y = R::ahead_y, P = R::ahead_p, U = R::unroll;
    const int nx = rw.nx, ny = rw.ny;
    const int rc = 2 * lane - D;                 // strip column of this lane's pair
    const int gcol = wrap(it.xs + rc, nx);
    const bool ocol = rc >= 0 && rc < it.ws;
    const double mcol = ocol ? 1.0 : 0.0;
    const int T_ = it.hb + 2 * D;
    const StenT<T> st = sten_as<T>(rw.st);
    T cc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cc[j] = static_cast<T>(rw.cc[j]);
    // lane parts of the offsets; the row parts are uniform
    const unsigned ycol = static_cast<unsigned>(gcol) * sizeof(Y0) / 2;
    const unsigned ocol8 = ocol ? static_cast<unsigned>(gcol) * 8u : kFar;
    const unsigned ocolT = ocol ? static_cast<unsigned>(gcol) * sizeof(T) : kFar;
    const unsigned row8 = static_cast<unsigned>(nx) * 8u, rowT = static_cast<unsigned>(nx) * sizeof(T);
    const unsigned rowY = static_cast<unsigned>(nx) * sizeof(Y0) / 2;
    const unsigned allY = rowY * static_cast<unsigned>(ny);

    P2<T> lc[D], lq[D];
#pragma unroll
    for (int j = 0; j < D; ++j) lc[j] = lq[j] = P2<T>{0, 0};
    // level 0, rows t .. t + Y - 1 (staged row t is y_m's row yb - D + t)
    Y0 yq[Y];
    unsigned yoff = static_cast<unsigned>(wrap(it.yb - D, ny)) * rowY;
#pragma unroll
    for (int i = 0; i < Y; ++i) {
        yq[i] = buf_ld<Y0>(rw.yin, ycol, yoff);
        yoff += rowY;
        if (yoff >= allY) yoff -= allY;
    }
    // the rows the outputs start from, rows t - D .. t - D + P - 1 (none
    // before step 2D is an output row)
    constexpr int KB = kShared ? 1 : K;
    double2 bq[KB][P];
#pragma unroll
    for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int i = 0; i < P; ++i) bq[k][i] = double2{0.0, 0.0};

    // step t, as sub-step u = t mod U of an unrolled block
    auto step = [&](const int u, const int t) __attribute__((always_inline)) {
        // level 0 at row t, and the load of row t + Y in its place
        P2<T> cur = as_t2<T>(yq[u % Y]);
        yq[u % Y] = buf_ld<Y0>(rw.yin, ycol, yoff);
        yoff += rowY;
        if (yoff >= allY) yoff -= allY;
        // output row t - D (band row t - 2D) starts from its loaded row;
        // row t - D + P is loaded in its place
        const int os = t - 2 * D, ol = os + P;
        const bool vs = os >= 0 && os < it.hb, vl = ol >= 0 && ol < it.hb;
        const unsigned so = vs ? static_cast<unsigned>(it.yb + os) * row8 : kFar;
        const unsigned lo = vl ? static_cast<unsigned>(it.yb + ol) * row8 : kFar;
        double2 b[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            b[k] = bq[k][u % P];
            bq[k][u % P] = buf_ld<double2, kNontemporal>(rw.base[k], ocol8 + lo, 0);
        }
        double2 p[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            p[k] = b[kShared ? 0 : k];
            if constexpr (kFirst) {
                p[k].x = rw.s0[k] * p[k].x;
                p[k].y = rw.s0[k] * p[k].y;
            }
        }
        const double mo = vs ? mcol : 0.0;
#pragma unroll
        for (int j = 1; j <= J; ++j) {
            // cur: level j-1 at row t-j+1; y: level j at row t-j
            const P2<T> y = stream_complete<T>(st, lq[j - 1], cur);
            lq[j - 1] = stream_partial<T>(st, cc[j - 1], lc[j - 1], cur);
            lc[j - 1] = cur;
            cur = y;
            // level j at row t - D
            P2<T> yr = y;
            if (j < D) {
                P2<T>* slot_r = ring + (R::base(j) + ((u - D) & (R::size(j) - 1))) * 64;
                P2<T>* slot_w = ring + (R::base(j) + ((u - j) & (R::size(j) - 1))) * 64;
                yr = slot_r[lane];
                slot_w[lane] = y;
            }
            const double2 y64 = as_d2<T>(yr);
            sy[j - 1] = fma(mo, y64.x * y64.x + y64.y * y64.y, sy[j - 1]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                p[k].x = fma(rw.dk[k][j], y64.x, p[k].x);
                p[k].y = fma(rw.dk[k][j], y64.y, p[k].y);
                sp[k][j - 1] = fma(mo, p[k].x * p[k].x + p[k].y * p[k].y, sp[k][j - 1]);
            }
        }
        // row t - D is complete: y_{m+D} and every output
        buf_st<P2<T>>(cur, rw.yout, ocolT + (vs ? static_cast<unsigned>(it.yb + os) * rowT : kFar));
#pragma unroll
        for (int k = 0; k < K; ++k) buf_st<double2, kNontemporal>(p[k], rw.pout[k], ocol8 + so);
    };
    // whole blocks of U steps as straight-line code (no branch between the
    // steps, so the waits for loads count exactly); the few steps past the
    // staged rows load rows that exist, store nothing and add nothing
    for (int t0 = 0; t0 < T_; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) step(u, t0 + u);
    }
}

// This wavefront's items of a ring window launch.
template <int K, int D, typename T, bool kFirst, bool kIn32, int J = D, bool kShared = false>
__device__ __forceinline__ void ring_items(const RingWin<K, D>& rw, const SweepArgs& a, const int wg, const int lane,
                                           double2* __restrict__ ring, double (&sy)[D], double (&sp)[K][D]) {
    const int items = a.tiles_x * a.tiles_y, G = a.nb * kStreamWaves;
    for (int i = stream_wave(wg, a.nb); i < items; i += G)
        ring_window_item<K, D, T, kFirst, kIn32, J, kShared>(
            rw, stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, strip_unit(a.nx, D)), lane,
            reinterpret_cast<P2<T>*>(ring), sy, sp);
}

// A re-execution (FP64 levels, not the first window) forms only the levels
// its outputs' terms need: J = jmax.
template <int K, int D, int J>
__device__ __forceinline__ void ring_redo(const int jmax, const RingWin<K, D>& rw, const SweepArgs& a, const int wg,
                                          const int lane, double2* __restrict__ ring, double (&sy)[D],
                                          double (&sp)[K][D]) {
    if constexpr (J < D) {
        if (jmax == J) {
            ring_items<K, D, double, false, false, J>(rw, a, wg, lane, ring, sy, sp);
            return;
        }
        ring_redo<K, D, J + 1>(jmax, rw, a, wg, lane, ring, sy, sp);
    } else {
        ring_items<K, D, double, false, false, D>(rw, a, wg, lane, ring, sy, sp);
    }
}

// The items of a ring window launch (this wavefront's share), with the
// launch's buffers and coefficients set up once.
// kLaunch0: launch 0, always the first window, neither re-executed nor
// copying, whose outputs all start from y_m: only that form is compiled.
template <int K, int D, bool F32, bool kLaunch0>
__device__ __forceinline__ void ring_windows(const SweepArgs& a, const WindowPlan<K>& w, const int wg, const int lane,
                                             double2* __restrict__ ring_mem, double (&sy)[D], double (&sp)[K][D]) {
    RingWin<K, D> rw;
    rw.nx = a.nx;
    rw.ny = a.ny;
    rw.st = Sten{a.aW, a.aE, a.aS, a.aN, a.aC, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < D; ++j) rw.cc[j] = a.aC - a.xi[w.m + j];
    const unsigned n = static_cast<unsigned>(a.nx) * static_cast<unsigned>(a.ny);
    const bool win32 = F32 && w.win32, in32 = F32 && w.in32, first = w.win == 0;
    rw.yin = make_rsrc(w.yin, n * (in32 ? 4u : 8u));
    rw.yout = make_rsrc(w.yout, (!w.redo && w.yout != nullptr) ? n * (win32 ? 4u : 8u) : 0u);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // the first window starts from p_0 = d_m y_m (also when it is
        // re-executed); a copy reads the window's own result
        const bool fk = first && !w.copy[k];
        const bool wr = w.nt[k] > 0 || w.copy[k];
        rw.s0[k] = fk ? a.coef[k * a.ld + w.m] : 1.0;
        rw.base[k] = make_rsrc(fk ? static_cast<const void*>(w.yin) : static_cast<const void*>(w.pin[k]),
                               (fk || wr) ? n * 8u : 0u);
        rw.pout[k] = make_rsrc(w.pout[k], wr ? n * 8u : 0u);
#pragma unroll
        for (int j = 1; j <= D; ++j) rw.dk[k][j] = j <= w.nt[k] ? a.coef[k * a.ld + w.m + j] : 0.0;
    }
    // this wavefront's rings, cleared once so that rows no output takes
    // (before step 2D of the first item) hold finite values
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    double2* ring = ring_mem + wave * Ring<D>::slots * 64;
#pragma unroll
    for (int i = 0; i < Ring<D>::slots; ++i) ring[i * 64 + lane] = double2{0.0, 0.0};
    if (win32) {
        if (first) ring_items<K, D, float, true, false>(rw, a, wg, lane, ring, sy, sp);
        else if (in32) ring_items<K, D, float, false, true>(rw, a, wg, lane, ring, sy, sp);
        else ring_items<K, D, float, false, false>(rw, a, wg, lane, ring, sy, sp);
    } else if (first) {
        if constexpr (kLaunch0) ring_items<K, D, double, true, false, D, true>(rw, a, wg, lane, ring, sy, sp);
        else ring_items<K, D, double, true, false>(rw, a, wg, lane, ring, sy, sp);
    } else if constexpr (!kLaunch0) {
        // a window in which one output still takes terms, or a re-execution
        // that recomputes one output and copies none, runs the one-output
        // form (the others' work is all masked: loads of nothing, products
        // by 0); its sums go to that output's place, the others' stay 0, and
        // every operation on that output is the same
        int nact = 0, kact = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (w.nt[k] > 0) {
                ++nact;
                kact = k;
            }
        bool copies = false;
#pragma unroll
        for (int k = 0; k < K; ++k) copies = copies || w.copy[k];
        if (w.redo && !(K > 1 && nact == 1 && !copies)) {
            ring_redo<K, D, 1>(w.jmax, rw, a, wg, lane, ring, sy, sp);
        } else if (K > 1 && nact == 1) {
            RingWin<1, D> r1;
            r1.nx = rw.nx;
            r1.ny = rw.ny;
            r1.st = rw.st;
#pragma unroll
            for (int j = 0; j < D; ++j) r1.cc[j] = rw.cc[j];
            r1.yin = rw.yin;
            r1.yout = rw.yout;
            r1.s0[0] = 1.0;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == kact) {
                    r1.base[0] = rw.base[k];
                    r1.pout[0] = rw.pout[k];
#pragma unroll
                    for (int j = 1; j <= D; ++j) r1.dk[0][j] = rw.dk[k][j];
                }
            double s1[1][D];
#pragma unroll
            for (int j = 0; j < D; ++j) s1[0][j] = 0.0;
            if (w.redo) ring_redo<1, D, 1>(w.jmax, r1, a, wg, lane, ring, sy, s1);
            else ring_items<1, D, double, false, false>(r1, a, wg, lane, ring, sy, s1);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (k == kact) sp[k][j] += s1[0][j];
        } else {
            ring_items<K, D, double, false, false>(rw, a, wg, lane, ring, sy, sp);
        }
    }
}

// Launch L of the window loop: a.tiles_x strips by a.tiles_y bands, a.nb
// workgroups of kStreamWaves wavefronts.  F32: FP32 sweeps (windows switch
// to FP32 levels on the device, window_enter; both precisions in one kernel).
template <int OP, int K, int D, bool F32, bool kLaunch0 = false>
__device__ __forceinline__ void leja_stream_body(const SweepArgs& a, const int L) {
    if (loop_ended(a.ctl)) return;
    const int wg = static_cast<int>(blockIdx.x);
    WindowPlan<K> w;
    if (!window_enter<OP, K, D, true, F32>(a, L, wg, nullptr, w)) return;
    double sy[D], sp[K][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sy[j] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sp[k][j] = 0.0;
    }
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int items = a.tiles_x * a.tiles_y, G = a.nb * kStreamWaves;
    if (w.jmax == 0) {
        // a re-execution with copies only, or nothing at all (the sums it
        // records are not read: the launch after a re-execution goes on
        // without a stop test)
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) any = any || w.copy[k];
        if (any)
            for (int i = stream_wave(wg, a.nb); i < items; i += G)
                stream_copy_item<K>(w, stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, strip_unit(a.nx, D)), lane,
                                    a.nx);
    } else if constexpr (kRingWindows<OP, D>) {
        __shared__ double2 ring_mem[kStreamWaves * Ring<D>::slots * 64];
        ring_windows<K, D, F32, kLaunch0>(a, w, wg, lane, ring_mem, sy, sp);
    } else {
        // the window's coefficients
        double dk[K][D + 1], cc[D];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j <= D; ++j) dk[k][j] = a.coef[k * a.ld + w.m + j];
        const double centre = OP == kOpBurgersJ ? a.kC : a.aC;
#pragma unroll
        for (int j = 0; j < D; ++j) cc[j] = centre - a.xi[w.m + j];
        const TileArgs<K> ta = tile_args<OP, K>(a);
        const int unit = strip_unit(a.nx, D);
        if (F32 && w.win32) {
            for (int i = stream_wave(wg, a.nb); i < items; i += G)
                stream_window_item<OP, K, D, float>(ta, w, a.u32, dk, cc,
                                                    stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, unit), lane, sy,
                                                    sp);
        } else {
            for (int i = stream_wave(wg, a.nb); i < items; i += G)
                stream_window_item<OP, K, D, double>(ta, w, a.u, dk, cc,
                                                     stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, unit), lane, sy,
                                                     sp);
        }
    }
    window_exit<K, D>(a, L, wg, sy, sp);
}

template <int OP, int K, int D, bool F32>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void leja_stream(SweepArgs a,
                                                                                                const int L) {
    leja_stream_body<OP, K, D, F32>(a, L);
}

// The same at one wavefront per SIMD (kDeepRing), with its registers; launch
// 0 (the first window) has a kernel of its own, since the registers of a
// kernel are allocated over all its forms and the first window's form,
// compiled beside the others, cost the full windows 12 % (and, in its
// general form with a start row per output, took half as long again as a
// full window itself).
template <int OP, int K, int D, bool F32>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void leja_stream_deep(
    SweepArgs a, const int L) {
    leja_stream_body<OP, K, D, F32>(a, L);
}

template <int OP, int K, int D, bool F32>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void leja_stream_deep_first(
    SweepArgs a) {
    leja_stream_body<OP, K, D, F32, true>(a, 0);
}

// ---------------------------------------------------------------------------
// Power iteration, up to DP sweeps per launch: level j = A^j (x / ||x||)
// formed by the same streaming (no shift), the sums of squares of every
// level recorded, the last level written; the next launch scales by its norm.
// The directions are those of the normalised iteration x_{k+1} = A x_k /
// ||A x_k||, and rho_hat = ||level nlev|| / ||level nlev-1|| of the last
// launch (level 0 has norm 1).  The host bounds nlev so that the unnormalised
// levels (at most rho^j) stay far from overflow.  With raw0 the first launch
// takes the start vector x as it is (levels A^j x, the same directions) and
// records ||x||^2 itself, which saves a pass over x; the final launch then
// reports a NaN estimate unless ||x||^2 lay in [1e-200, 1e20], where the
// unscaled levels keep the margin of the scaled ones, and the host repeats
// the iteration with x scaled first.
// Partial sums: the start vector's (power_norm_kernel, or launch 0 with
// raw0) at partials[nb + i], launch b's at partials[2 nb + (b & 1) nb DP +
// i DP + j].
// ---------------------------------------------------------------------------

// One item of a power launch that makes DP levels: level 0 (row t of `in`,
// scaled by s) is loaded four steps ahead through a buffer resource and
// every step issues the same memory operations (rows and lanes outside the
// item's output get offsets past the end), so no step waits for the load
// it has just issued.  Steps run in whole blocks of U; the few past the
// staged rows store nothing and add nothing.  kLevel0: also the sum of
// squares of level 0 on the item's output points, into sy0.
template <int DP, bool kLevel0>
__device__ __forceinline__ void stream_power_item(const StenT<double>& st, const double centre, const int nx,
                                                  const int ny, const Rsrc in, const Rsrc out, const double s,
                                                  const StreamItem it, const int lane, double (&sy)[DP],
                                                  double& sy0) {
    constexpr int Y = 4, U = 4;   // U: a multiple of Y and of 2 (the roles of lc and lq)
    const int rc = 2 * lane - DP;
    const int gcol = wrap(it.xs + rc, nx);
    const bool ocol = rc >= 0 && rc < it.ws;
    const double mcol = ocol ? 1.0 : 0.0;
    const int T = it.hb + 2 * DP;
    const unsigned col8 = static_cast<unsigned>(gcol) * 8u, ocol8 = ocol ? col8 : kFar;
    const unsigned row8 = static_cast<unsigned>(nx) * 8u, all8 = row8 * static_cast<unsigned>(ny);
    double2 lc[DP], lq[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) lc[j] = lq[j] = double2{0.0, 0.0};
    double2 yq[Y];
    unsigned yoff = static_cast<unsigned>(wrap(it.yb - DP, ny)) * row8;
#pragma unroll
    for (int i = 0; i < Y; ++i) {
        yq[i] = buf_ld<double2>(in, col8, yoff);
        yoff += row8;
        if (yoff >= all8) yoff -= all8;
    }
    for (int t0 = 0; t0 < T; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u;
            double2 cur;
            cur.x = s * yq[u % Y].x;
            cur.y = s * yq[u % Y].y;
            yq[u % Y] = buf_ld<double2>(in, col8, yoff);
            yoff += row8;
            if (yoff >= all8) yoff -= all8;
            if constexpr (kLevel0) {
                const int r0 = t - DP;
                sy0 = fma(r0 >= 0 && r0 < it.hb ? mcol : 0.0, cur.x * cur.x + cur.y * cur.y, sy0);
            }
#pragma unroll
            for (int j = 1; j <= DP; ++j) {
                const double2 y = stream_complete<double>(st, lq[j - 1], cur);
                lq[j - 1] = stream_partial<double>(st, centre, lc[j - 1], cur);
                lc[j - 1] = cur;
                cur = y;
                // level j at row t - j, band row t - j - DP
                const int r = t - j - DP;
                const bool vr = r >= 0 && r < it.hb;
                sy[j - 1] = fma(vr ? mcol : 0.0, y.x * y.x + y.y * y.y, sy[j - 1]);
                if (j == DP) buf_st<double2>(y, out, ocol8 + (vr ? static_cast<unsigned>(it.yb + r) * row8 : kFar));
            }
        }
    }
}

// Any number of levels nlev <= DP (the last launch of a power iteration
// whose sweeps are not a multiple of DP).
template <int DP>
__device__ __forceinline__ void stream_power_item_any(const Sten& st, const int nx, const int ny,
                                                  const double* __restrict__ in, double* __restrict__ out,
                                                  const double s, const int nlev, const StreamItem it, const int lane,
                                                  double (&sy)[DP]) {
    const int rc = 2 * lane - DP;
    const int gcol = wrap(it.xs + rc, nx);
    const bool ocol = rc >= 0 && rc < it.ws;
    const int T = it.hb + 2 * DP;
    const StenT<double> stt = sten_as<double>(st);
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
                const double2 y = stream_complete<double>(stt, lq[j - 1], cur);
                lq[j - 1] = stream_partial<double>(stt, st.c4, lc[j - 1], cur);
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
// of launch b - 1 (which made prev levels) or of the start vector (b = 0:
// unscaled with raw0, which needs nlev = DP).
template <int DP>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void power_stream(
    PowerArgs a, const double* in, double* out, const int b, const int nlev, const int prev, const int raw0) {
    const int wg = static_cast<int>(blockIdx.x);
    const bool lev0 = b == 0 && raw0 != 0;
    double scale = 1.0;
    if (b == 0) {
        if (!lev0) {
            double tot[1];
            sum_partials<1>(a.partials + a.nb, a.nb, tot);
            scale = 1.0 / sqrt(tot[0]);
        }
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
    const StenT<double> st{a.cW, a.cE, a.cS, a.cN};
    double sy[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) sy[j] = 0.0;
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int items = a.tiles_x * a.tiles_y, G = a.nb * kStreamWaves;
    const int unit = strip_unit(a.nx, DP);
    double sy0 = 0.0;
    if (nl == DP) {
        const unsigned bytes = static_cast<unsigned>(a.nx) * static_cast<unsigned>(a.ny) * 8u;
        const Rsrc rin = make_rsrc(in, bytes), rout = make_rsrc(out, bytes);
        if (lev0) {
            for (int i = stream_wave(wg, a.nb); i < items; i += G)
                stream_power_item<DP, true>(st, a.cC, a.nx, a.ny, rin, rout, scale,
                                            stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, unit), lane, sy, sy0);
        } else {
            for (int i = stream_wave(wg, a.nb); i < items; i += G)
                stream_power_item<DP, false>(st, a.cC, a.nx, a.ny, rin, rout, scale,
                                             stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, unit), lane, sy, sy0);
        }
    } else {
        const Sten sa{a.cW, a.cE, a.cS, a.cN, a.cC, 0.0, 0.0, 0.0, 0.0};
        for (int i = stream_wave(wg, a.nb); i < items; i += G)
            stream_power_item_any<DP>(sa, a.nx, a.ny, in, out, scale, nl,
                                      stream_geom(i, a.nx, a.ny, a.tiles_x, a.tiles_y, unit), lane, sy);
    }
    block_sum<DP>(sy);
    if (lev0) {
        double s0[1] = {sy0};
        block_sum<1>(s0);
        sy0 = s0[0];
    }
    if (flat_tid() == 0) {
        double* __restrict__ Pp = a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * DP + static_cast<long>(wg) * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) Pp[j] = sy[j];
        if (lev0) a.partials[a.nb + wg] = sy0;
    }
}

// rho_hat = ||level nlev|| / ||level nlev-1|| of the last launch b; NaN
// after an unscaled first launch (raw0) whose ||x||^2 left [1e-200, 1e20]
template <int DP>
__global__ __launch_bounds__(kBlockThreads) void power_stream_final(PowerArgs a, const int b, const int nlev,
                                                                    const int raw0) {
    double tot[DP];
    sum_partials<DP>(a.partials + 2L * a.nb + static_cast<long>(b & 1) * a.nb * DP, a.nb, tot);
    double x2[1] = {1.0};
    if (raw0) sum_partials<1>(a.partials + a.nb, a.nb, x2);
    if (flat_tid() == 0) {
        double last = 0.0, prev = 1.0;
#pragma unroll
        for (int j = 0; j < DP; ++j) {
            if (j == nlev - 1) last = tot[j];
            if (j == nlev - 2) prev = tot[j];
        }
        const bool safe = x2[0] >= 1e-200 && x2[0] <= 1e20;
        a.ctl->rho = safe ? sqrt(last / prev) : __builtin_nan("");
    }
}

// The register-marching window kernels there are: the five-point
// diffusion-advection operator at depth 4 (K <= 4), 6 (K <= 3) and 8 (K <= 3)
// in FP64, and the Burgers Jacobian at depth 4 (K <= 2) and 6 (K = 1); FP32
// sweeps for K <= 2 at depths 4 and 6 (K = 1) of both operators.
#define LX_STREAM_KERNELS(X)                                                                              \
    X(kOpDiffAdv, 1, 4, false) X(kOpDiffAdv, 2, 4, false) X(kOpDiffAdv, 3, 4, false)                      \
    X(kOpDiffAdv, 4, 4, false) X(kOpDiffAdv, 1, 6, false) X(kOpDiffAdv, 2, 6, false)                      \
    X(kOpDiffAdv, 3, 6, false) X(kOpDiffAdv, 1, 8, false) X(kOpDiffAdv, 2, 8, false)                      \
    X(kOpDiffAdv, 3, 8, false) X(kOpBurgersJ, 1, 4, false) X(kOpBurgersJ, 2, 4, false)                    \
    X(kOpBurgersJ, 1, 6, false) X(kOpDiffAdv, 1, 4, true) X(kOpDiffAdv, 2, 4, true)                       \
    X(kOpDiffAdv, 1, 6, true) X(kOpBurgersJ, 1, 4, true) X(kOpBurgersJ, 2, 4, true)                       \
    X(kOpBurgersJ, 1, 6, true)

// the kernel of a (operator, K, depth, precision) combination, and its launch
template <int OP, int K, int D, bool F32>
const void* stream_fn() {
    if constexpr (kDeepRing<OP, D>) return reinterpret_cast<const void*>(leja_stream_deep<OP, K, D, F32>);
    else return reinterpret_cast<const void*>(leja_stream<OP, K, D, F32>);
}

template <int OP, int K, int D, bool F32>
void stream_launch(const SweepArgs& a, const int L, hipStream_t s) {
    if constexpr (kDeepRing<OP, D>) {
        if (L == 0) hipLaunchKernelGGL((leja_stream_deep_first<OP, K, D, F32>), dim3(a.nb), dim3(kBlockThreads), 0, s, a);
        else hipLaunchKernelGGL((leja_stream_deep<OP, K, D, F32>), dim3(a.nb), dim3(kBlockThreads), 0, s, a, L);
    } else
        hipLaunchKernelGGL((leja_stream<OP, K, D, F32>), dim3(a.nb), dim3(kBlockThreads), 0, s, a, L);
}

const void* stream_kernel(int op, int K, int depth, bool f32) {
#define LX_STREAM_PICK(O, KK, DD, F)                                                    \
    if (op == (O) && K == (KK) && depth == (DD) && f32 == (F)) return stream_fn<(O), (KK), (DD), (F)>();
    LX_STREAM_KERNELS(LX_STREAM_PICK)
#undef LX_STREAM_PICK
    return nullptr;
}

}  // namespace

int stream_strips(int nx, int depth) {
    const int unit = strip_unit(nx, depth);
    const int out_units = (128 - 2 * depth) / unit;   // column units a strip outputs
    return ((nx / unit) + out_units - 1) / out_units;
}

bool stream_has(int op, int K, int depth, bool fp32) { return stream_kernel(op, K, depth, fp32) != nullptr; }

hipError_t launch_leja_stream(int op, int K, int depth, bool fp32, const SweepArgs& a, int L, hipStream_t s) {
    if (!stream_has(op, K, depth, fp32) || a.nb < 1 || a.nx % 2 != 0 || a.nx < depth || a.ny < depth)
        return hipErrorInvalidValue;
    if (op == kOpBurgersJ && (a.u == nullptr || (fp32 && a.u32 == nullptr))) return hipErrorInvalidValue;
    if (a.tiles_x != stream_strips(a.nx, depth) || a.tiles_y < 1 || a.tiles_y > a.ny) return hipErrorInvalidValue;
    if (static_cast<long>(a.nx) * a.ny * 8 > static_cast<long>(kFar)) return hipErrorInvalidValue;
#define LX_STREAM_LAUNCH(O, KK, DD, F)                                                                         \
    if (op == (O) && K == (KK) && depth == (DD) && fp32 == (F)) {                                              \
        stream_launch<(O), (KK), (DD), (F)>(a, L, s);                                                          \
        return hipGetLastError();                                                                              \
    }
    LX_STREAM_KERNELS(LX_STREAM_LAUNCH)
#undef LX_STREAM_LAUNCH
    return hipErrorInvalidValue;
}

int stream_resident(int op, int K, int depth, bool fp32, int power) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void* k = power ? reinterpret_cast<const void*>(power_stream<kPowerStreamDepth>)
                          : stream_kernel(op, K, depth, fp32);
    if (k == nullptr) return 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlockThreads, 0);
    return e == hipSuccess ? per_cu * cus : 0;
}

hipError_t launch_power_stream(const PowerArgs& a, const double* in, double* out, int b, int nlev, int prev,
                               bool raw0, hipStream_t s) {
    constexpr int DP = kPowerStreamDepth;
    if (a.nb < 1 || a.nx % 2 != 0 || a.nx < DP || a.ny < DP || nlev < 1 || nlev > DP || prev < 1 || prev > DP)
        return hipErrorInvalidValue;
    if (raw0 && b == 0 && nlev != DP) return hipErrorInvalidValue;
    if (a.tiles_x != stream_strips(a.nx, DP) || a.tiles_y < 1 || a.tiles_y > a.ny) return hipErrorInvalidValue;
    if (static_cast<long>(a.nx) * a.ny * 8 > static_cast<long>(kFar)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((power_stream<DP>), dim3(a.nb), dim3(kBlockThreads), 0, s, a, in, out, b, nlev, prev,
                       raw0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_power_stream_final(const PowerArgs& a, int b, int nlev, bool raw0, hipStream_t s) {
    hipLaunchKernelGGL((power_stream_final<kPowerStreamDepth>), dim3(1), dim3(kBlockThreads), 0, s, a, b, nlev,
                       raw0 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lx
