// Device building blocks of the Leja sweeps, shared by the single-grid
// kernels (kernels.hip) and the batched kernels (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "lx_device.h"

namespace lx {
namespace dev {


// A device pointer marked as global memory.  Pointers read from memory
// (the batched kernels keep their arguments in LDS) are generic to the
// compiler, which then accesses through them with flat instructions: these
// count on both the vector-memory and the LDS counters, so every wait for
// an LDS read also waits for the global loads in flight.
template <typename T>
__device__ __forceinline__ T* gptr(T* p) {
    using G = __attribute__((address_space(1))) T*;
    return (T*)((G)(reinterpret_cast<unsigned long long>(p)));
}

__device__ __forceinline__ int wrap(int r, int n) {
    if (r < 0) r += n;
    else if (r >= n) r -= n;
    if (r >= n) r %= n;      // only when a tile is taller than the grid
    return r;
}

// Calls f(tile) for the tiles of this workgroup.  With nb a multiple of 8,
// workgroup b runs on XCD b % 8 and takes every (nb/8)-th tile of that XCD's
// contiguous band, so that concurrently running workgroups of one XCD work
// on neighbouring tiles.
template <typename F>
__device__ __forceinline__ void for_each_tile(int T, int nb, F&& f) {
    const int b = static_cast<int>(blockIdx.x);
    if (nb >= 8 && (nb & 7) == 0) {
        const int x = b & 7, j = b >> 3, nbx = nb >> 3;
        const int lo = static_cast<int>((static_cast<long>(x) * T) >> 3);
        const int hi = static_cast<int>((static_cast<long>(x + 1) * T) >> 3);
        for (int t = lo + j; t < hi; t += nbx) f(t);
    } else {
        for (int t = b; t < T; t += nb) f(t);
    }
}

__device__ __forceinline__ int flat_tid() { return threadIdx.x + threadIdx.y * blockDim.x; }

// Workgroup j of nb takes the contiguous tiles [T j / nb, T (j+1) / nb):
// consecutive tiles are neighbours, so the halo rows a tile reads were
// fetched by the same workgroup (and its XCD's L2) just before.
template <typename F>
__device__ __forceinline__ void for_tile_band(int T, int nb, int j, F&& f) {
    const int lo = static_cast<int>((static_cast<long>(j) * T) / nb);
    const int hi = static_cast<int>((static_cast<long>(j + 1) * T) / nb);
    for (int t = lo; t < hi; ++t) f(t);
}
__device__ __forceinline__ int block_threads() { return blockDim.x * blockDim.y; }

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

template <int V, typename T, typename A>
__device__ __forceinline__ void ldv(const T* __restrict__ p, A (&o)[V]) {
    if constexpr (V == 2) {
        const auto t = *reinterpret_cast<const typename Pair<T>::type*>(p);
        o[0] = static_cast<A>(t.x);
        o[1] = static_cast<A>(t.y);
    } else {
        o[0] = static_cast<A>(p[0]);
    }
}

template <int V, typename T>
__device__ __forceinline__ void stv(T* __restrict__ p, const T (&o)[V]) {
    if constexpr (V == 2) {
        typename Pair<T>::type t;
        t.x = o[0];
        t.y = o[1];
        *reinterpret_cast<typename Pair<T>::type*>(p) = t;
    } else {
        p[0] = o[0];
    }
}

// Streaming (nontemporal) variants for the outputs p_k, which each launch
// reads and writes once.  The hint keeps them from displacing the basis
// vector in the caches: on MI355X the basis vector of a 4096^2 grid
// (134 MB) then stays in the 256 MB Infinity Cache from the launch that
// writes it to the launch that reads it.  Measured at 4096^2 with three
// outputs: 105 us per iteration without hints, 92 with hints on p and the
// basis vector, 79 with hints on p only.
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };

template <int V, typename T, typename A>
__device__ __forceinline__ void ldv_nt(const T* __restrict__ p, A (&o)[V]) {
    if constexpr (V == 2) {
        const auto t = __builtin_nontemporal_load(reinterpret_cast<const typename Vec2<T>::type*>(p));
        o[0] = static_cast<A>(t.x);
        o[1] = static_cast<A>(t.y);
    } else {
        o[0] = static_cast<A>(__builtin_nontemporal_load(p));
    }
}

template <int V, typename T>
__device__ __forceinline__ void stv_nt(T* __restrict__ p, const T (&o)[V]) {
    if constexpr (V == 2) {
        typename Vec2<T>::type t;
        t.x = o[0];
        t.y = o[1];
        __builtin_nontemporal_store(t, reinterpret_cast<typename Vec2<T>::type*>(p));
    } else {
        __builtin_nontemporal_store(o[0], p);
    }
}

// Sums NV values over the workgroup in a fixed order (butterfly within each
// 64-lane wavefront, then wavefronts in index order); every thread receives
// the result.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NV][kBlockThreads / 64];
    __shared__ double out[NV];
    const int tid = flat_tid();
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        v[q] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q][wid] = v[q];
    }
    __syncthreads();
    if (tid < NV) {
        const int nw = (block_threads() + 63) >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[tid][w];
        out[tid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = out[q];
    __syncthreads();
}

// Whether the loop behind `ctl` has ended, read by one lane for the whole
// workgroup: workgroup 0 of the same launch may publish the flag while this
// workgroup starts, and all its wavefronts must take the same branch since
// they meet at barriers later.
// The final state of a loop, into slot[2] and, when the caller gave one,
// into its host-visible copy (pinned host memory, written through to
// system scope), which the host may read as soon as it sees done = 1, while
// the launch still runs: the word holding `done` goes last, after a
// system-scope fence.  The copy goes word by word from slot[2], so that the
// state needs no private memory.
__device__ __forceinline__ void publish_final(LoopCtl* ctl, SweepState* pub, const SweepState& st) {
    ctl->slot[2] = st;
    if (pub != nullptr) {
        static_assert(sizeof(SweepState) % sizeof(unsigned long long) == 0, "SweepState in 8-byte words");
        constexpr int kWords = static_cast<int>(sizeof(SweepState) / sizeof(unsigned long long));
        constexpr int kDone = static_cast<int>(offsetof(SweepState, done) / sizeof(unsigned long long));
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(&ctl->slot[2]);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(pub);
        for (int i = 0; i < kWords; ++i)
            if (i != kDone) dst[i] = src[i];
        __threadfence_system();
        dst[kDone] = src[kDone];
        __threadfence_system();
    }
}

__device__ __forceinline__ bool loop_ended(const LoopCtl* ctl) {
    __shared__ int s_end;
    if (flat_tid() == 0) s_end = ctl->slot[2].done;
    __syncthreads();
    return s_end != 0;
}

// Adds the nb partial records of NV values written by the previous launch,
// in workgroup-index order per lane and then block_sum's fixed tree: every
// workgroup of the grid obtains bitwise the same totals.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ P, int nb, double (&tot)[NV]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) tot[q] = 0.0;
    for (int b = flat_tid(); b < nb; b += block_threads()) {
#pragma unroll
        for (int q = 0; q < NV; ++q) tot[q] += P[b * NV + q];
    }
    block_sum<NV>(tot);
}

// ---------------------------------------------------------------------------
// the stencils, with every product and sum in a fixed order (explicit FMAs,
// no contraction left to the compiler), so that all kernels compute the
// same bits from the same inputs
// ---------------------------------------------------------------------------

// diffusion-advection: cW W + cE E + cS S + cN N + cC C
template <typename T>
__device__ __forceinline__ T stencil_da(T cW, T cE, T cS, T cN, T cC, T W, T E, T S, T N, T C) {
#pragma clang fp contract(off)
    return fma(cN, N, fma(cS, S, fma(cE, E, fma(cW, W, cC * C))));
}

// radius-2 cross stencil (diffusion + third-order upwind advection): the
// five-point part, then the second neighbours W2, E2, S2, N2
template <typename T>
__device__ __forceinline__ T stencil_d3(T cW, T cE, T cS, T cN, T cC, T cW2, T cE2, T cS2, T cN2, T W, T E, T S, T N,
                                        T C, T W2, T E2, T S2, T N2) {
#pragma clang fp contract(off)
    T r = fma(cN, N, fma(cS, S, fma(cE, E, fma(cW, W, cC * C))));
    r = fma(cW2, W2, r);
    r = fma(cE2, E2, r);
    r = fma(cS2, S2, r);
    return fma(cN2, N2, r);
}

// Burgers Jacobian: kx (E + W) + ky (N + S) - gx (uE E - uW W) - gy (uN N - uS S) + kc C
template <typename T>
__device__ __forceinline__ T stencil_bu(T kx, T ky, T gx, T gy, T kc, T W, T E, T S, T N, T C, T uW, T uE, T uS,
                                        T uN) {
#pragma clang fp contract(off)
    const T ax = fma(uE, E, -(uW * W));
    const T ay = fma(uN, N, -(uS * S));
    T r = kc * C;
    r = fma(kx, E + W, r);
    r = fma(ky, N + S, r);
    r = fma(-gx, ax, r);
    return fma(-gy, ay, r);
}

// ---------------------------------------------------------------------------
// Leja sweep
// ---------------------------------------------------------------------------

template <int OP, int K, int RY, int V, typename TI, typename TO, typename AT>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const int m, const int (&act)[K],
                                           double& sy, double (&sp)[K], const int tile) {
    const int nx = a.nx, ny = a.ny;
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int col = (tile_x * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) * V;
    const bool colok = col < nx;
    const int c0 = colok ? col : 0;
    const int cl = (c0 == 0) ? nx - 1 : c0 - 1;
    const int cr = (c0 + V >= nx) ? c0 + V - nx : c0 + V;
    // second neighbours of the radius-2 stencil (nx >= 4)
    const int cl2 = wrap(c0 - 2, nx), cr2 = wrap(c0 + V + 1, nx);
    const int row0 = tile_y * static_cast<int>(blockDim.y) * RY + static_cast<int>(threadIdx.y) * RY;

    const TI* __restrict__ yin;
    if constexpr (sizeof(TI) == sizeof(double)) {
        yin = gptr((m == 0) ? reinterpret_cast<const TI*>(a.v) : static_cast<const TI*>(a.ybuf[(m - 1) & 1]));
    } else {
        yin = gptr(static_cast<const TI*>(a.ybuf[(m - 1) & 1]));
    }
    TO* __restrict__ yout = gptr(static_cast<TO*>(a.ybuf[m & 1]));

    double* __restrict__ pk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pk[k] = gptr(a.p[k]);
    const double* __restrict__ uu = gptr(a.u);
    const float* __restrict__ uu32 = gptr(a.u32);
    const double xim = gptr(a.xi)[m];
    double dn1[K], d0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dn1[k] = gptr(a.coef)[k * a.ld + m + 1];
        d0[k] = gptr(a.coef)[k * a.ld];
    }

    AT up[V], cen[V], dn[V];
    AT uup[V], ucen[V], udn[V];
    AT up2[V], dn2[V];       // radius-2 stencil: rows two below and two above
    ldv<V>(yin + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, up);
    ldv<V>(yin + static_cast<long>(wrap(row0, ny)) * nx + c0, cen);
    if constexpr (OP == kOpDiffAdv3) {
        ldv<V>(yin + static_cast<long>(wrap(row0 - 2, ny)) * nx + c0, up2);
        ldv<V>(yin + static_cast<long>(wrap(row0 + 1, ny)) * nx + c0, dn);
    }
    if constexpr (OP == kOpBurgersJ) {
        if constexpr (sizeof(AT) == sizeof(double)) {
            ldv<V>(uu + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
            ldv<V>(uu + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
        } else {
            ldv<V>(uu32 + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
            ldv<V>(uu32 + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
        }
    }

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int row = row0 + r;
        const bool ok = colok && row < ny;
        const long rw = wrap(row, ny);
        const long rn = wrap(row + 1, ny);
        if constexpr (OP == kOpDiffAdv3) {
            ldv<V>(yin + static_cast<long>(wrap(row + 2, ny)) * nx + c0, dn2);
        } else {
            ldv<V>(yin + rn * nx + c0, dn);
        }
        const AT left = static_cast<AT>(yin[rw * nx + cl]);
        const AT right = static_cast<AT>(yin[rw * nx + cr]);
        AT o[V];
        if constexpr (OP == kOpDiffAdv3) {
            const AT left2 = static_cast<AT>(yin[rw * nx + cl2]);
            const AT right2 = static_cast<AT>(yin[rw * nx + cr2]);
            const AT aE = static_cast<AT>(a.aE), aW = static_cast<AT>(a.aW);
            const AT aN = static_cast<AT>(a.aN), aS = static_cast<AT>(a.aS);
            const AT aE2 = static_cast<AT>(a.aE2), aW2 = static_cast<AT>(a.aW2);
            const AT aN2 = static_cast<AT>(a.aN2), aS2 = static_cast<AT>(a.aS2);
            const AT ac = static_cast<AT>(a.aC - xim);
            if constexpr (V == 2) {
                o[0] = stencil_d3(aW, aE, aS, aN, ac, aW2, aE2, aS2, aN2, left, cen[1], up[0], dn[0], cen[0], left2,
                                  right, up2[0], dn2[0]);
                o[1] = stencil_d3(aW, aE, aS, aN, ac, aW2, aE2, aS2, aN2, cen[0], right, up[1], dn[1], cen[1], left,
                                  right2, up2[1], dn2[1]);
            } else {
                o[0] = stencil_d3(aW, aE, aS, aN, ac, aW2, aE2, aS2, aN2, left, right, up[0], dn[0], cen[0], left2,
                                  right2, up2[0], dn2[0]);
            }
        } else if constexpr (OP == kOpDiffAdv) {
            const AT aE = static_cast<AT>(a.aE), aW = static_cast<AT>(a.aW);
            const AT aN = static_cast<AT>(a.aN), aS = static_cast<AT>(a.aS);
            const AT ac = static_cast<AT>(a.aC - xim);
            if constexpr (V == 2) {
                o[0] = stencil_da(aW, aE, aS, aN, ac, left, cen[1], up[0], dn[0], cen[0]);
                o[1] = stencil_da(aW, aE, aS, aN, ac, cen[0], right, up[1], dn[1], cen[1]);
            } else {
                o[0] = stencil_da(aW, aE, aS, aN, ac, left, right, up[0], dn[0], cen[0]);
            }
        } else {
            const AT kx = static_cast<AT>(a.kx), ky = static_cast<AT>(a.ky);
            const AT gx = static_cast<AT>(a.gx), gy = static_cast<AT>(a.gy);
            const AT kc = static_cast<AT>(a.kC - xim);
            AT ul, ur;
            if constexpr (sizeof(AT) == sizeof(double)) {
                ldv<V>(uu + rn * nx + c0, udn);
                ul = uu[rw * nx + cl];
                ur = uu[rw * nx + cr];
            } else {
                ldv<V>(uu32 + rn * nx + c0, udn);
                ul = uu32[rw * nx + cl];
                ur = uu32[rw * nx + cr];
            }
            if constexpr (V == 2) {
                o[0] = stencil_bu(kx, ky, gx, gy, kc, left, cen[1], up[0], dn[0], cen[0], ul, ucen[1], uup[0], udn[0]);
                o[1] = stencil_bu(kx, ky, gx, gy, kc, cen[0], right, up[1], dn[1], cen[1], ucen[0], ur, uup[1], udn[1]);
            } else {
                o[0] = stencil_bu(kx, ky, gx, gy, kc, left, right, up[0], dn[0], cen[0], ul, ur, uup[0], udn[0]);
            }
        }
        TO ot[V];
        double od[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            ot[i] = static_cast<TO>(o[i]);
            od[i] = static_cast<double>(ot[i]);
        }
        const long idx = rw * nx + c0;
        if (ok) {
            stv<V>(yout + idx, ot);
#pragma unroll
            for (int i = 0; i < V; ++i) sy += od[i] * od[i];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!act[k]) continue;
            double pv[V];
            if (m == 0) {
                // p_0 = d_0 y_0; y_0 = v is the centre row
#pragma unroll
                for (int i = 0; i < V; ++i) pv[i] = d0[k] * static_cast<double>(cen[i]);
            } else {
                ldv_nt<V>(pk[k] + idx, pv);
            }
#pragma unroll
            for (int i = 0; i < V; ++i) pv[i] = fma(dn1[k], od[i], pv[i]);
            if (ok) {
                stv_nt<V>(pk[k] + idx, pv);
#pragma unroll
                for (int i = 0; i < V; ++i) sp[k] += pv[i] * pv[i];
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            if constexpr (OP == kOpDiffAdv3) up2[i] = up[i];
            up[i] = cen[i];
            cen[i] = dn[i];
            if constexpr (OP == kOpDiffAdv3) dn[i] = dn2[i];
            if constexpr (OP == kOpBurgersJ) {
                uup[i] = ucen[i];
                ucen[i] = udn[i];
            }
        }
    }
}

// Stop rule (Sec. 2.2) after sweep m-1, from the grid totals of its partial
// sums: the state entering sweep m.  tot = {sum y_m^2, sum p_k^2 ...}.
template <int K, bool FP32>
__device__ __forceinline__ SweepState decide(const SweepArgs& a, const LoopCtl& ctl, const SweepState& prev,
                                             const int m, const double (&tot)[1 + K]) {
    SweepState nx = prev;
    nx.iter = m;
    nx.n_fp32 = prev.n_fp32 + prev.out32;
    nx.in32 = prev.out32;
    const double ynorm = sqrt(tot[0]) * a.inv_sqrtN;
    nx.ynorm = ynorm;
    bool nonfinite = !isfinite(ynorm);
    bool any_active = false, all_small = true;
    const double rtol = ctl.rtol, atol = ctl.atol, sw = ctl.fp32_switch;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!prev.active[k]) continue;
        const double pn = sqrt(tot[1 + k]) * a.inv_sqrtN;
        const double e = fabs(gptr(a.coef)[k * a.ld + m]) * ynorm;
        const double thr = rtol * pn + atol;
        nx.err[k] = e;
        nx.pnorm[k] = pn;
        if (!isfinite(pn) || !isfinite(e)) {
            nonfinite = true;
            nx.active[k] = 0;
            nx.iters[k] = m;
        } else if (e <= thr) {
            nx.active[k] = 0;
            nx.iters[k] = m;
        } else {
            any_active = true;
            if (!(e <= sw * thr)) all_small = false;
        }
    }
    if (FP32 && !prev.out32 && any_active && all_small && sw >= 0.0) nx.out32 = 1;
    if (nonfinite) {
        nx.status = 4;  // LX_ENONFINITE
        nx.done = 1;
    } else if (!any_active) {
        nx.status = 0;
        nx.done = 1;
    } else if (m >= ctl.max_iters) {
        nx.status = 3;  // LX_ENOTCONV
        nx.done = 1;
    }
    return nx;
}

// ---------------------------------------------------------------------------
// power iteration: w_{k+1} = (A w_k) / ||w_k||; ||w_k|| comes from the
// partial sums of the previous launch (the start-vector norm for k = 0)
// ---------------------------------------------------------------------------

template <int OP, int RY, int V>
__device__ __forceinline__ void power_tile(const PowerArgs& a, const double s, double& acc, const int tile) {
    const int nx = a.nx, ny = a.ny;
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int col = (tile_x * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) * V;
    const bool colok = col < nx;
    const int c0 = colok ? col : 0;
    const int cl = (c0 == 0) ? nx - 1 : c0 - 1;
    const int cr = (c0 + V >= nx) ? c0 + V - nx : c0 + V;
    // second neighbours of the radius-2 stencil (nx >= 4)
    const int cl2 = wrap(c0 - 2, nx), cr2 = wrap(c0 + V + 1, nx);
    const int row0 = tile_y * static_cast<int>(blockDim.y) * RY + static_cast<int>(threadIdx.y) * RY;
    const double* __restrict__ in = a.in;
    const double* __restrict__ uu = a.u;
    double* __restrict__ out = a.out;

    double up[V], cen[V], dn[V], uup[V], ucen[V], udn[V], up2[V], dn2[V];
    ldv<V>(in + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, up);
    ldv<V>(in + static_cast<long>(wrap(row0, ny)) * nx + c0, cen);
    if constexpr (OP == kOpDiffAdv3) {
        ldv<V>(in + static_cast<long>(wrap(row0 - 2, ny)) * nx + c0, up2);
        ldv<V>(in + static_cast<long>(wrap(row0 + 1, ny)) * nx + c0, dn);
    }
    if constexpr (OP == kOpBurgersJ) {
        ldv<V>(uu + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
        ldv<V>(uu + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int row = row0 + r;
        const bool ok = colok && row < ny;
        const long rw = wrap(row, ny);
        const long rn = wrap(row + 1, ny);
        if constexpr (OP == kOpDiffAdv3) {
            ldv<V>(in + static_cast<long>(wrap(row + 2, ny)) * nx + c0, dn2);
        } else {
            ldv<V>(in + rn * nx + c0, dn);
        }
        const double left = in[rw * nx + cl], right = in[rw * nx + cr];
        double o[V];
        if constexpr (OP == kOpDiffAdv3) {
            const double left2 = in[rw * nx + cl2], right2 = in[rw * nx + cr2];
            if constexpr (V == 2) {
                o[0] = stencil_d3(a.cW, a.cE, a.cS, a.cN, a.cC, a.cW2, a.cE2, a.cS2, a.cN2, left, cen[1], up[0], dn[0],
                                  cen[0], left2, right, up2[0], dn2[0]);
                o[1] = stencil_d3(a.cW, a.cE, a.cS, a.cN, a.cC, a.cW2, a.cE2, a.cS2, a.cN2, cen[0], right, up[1], dn[1],
                                  cen[1], left, right2, up2[1], dn2[1]);
            } else {
                o[0] = stencil_d3(a.cW, a.cE, a.cS, a.cN, a.cC, a.cW2, a.cE2, a.cS2, a.cN2, left, right, up[0], dn[0],
                                  cen[0], left2, right2, up2[0], dn2[0]);
            }
        } else if constexpr (OP == kOpDiffAdv) {
            if constexpr (V == 2) {
                o[0] = stencil_da(a.cW, a.cE, a.cS, a.cN, a.cC, left, cen[1], up[0], dn[0], cen[0]);
                o[1] = stencil_da(a.cW, a.cE, a.cS, a.cN, a.cC, cen[0], right, up[1], dn[1], cen[1]);
            } else {
                o[0] = stencil_da(a.cW, a.cE, a.cS, a.cN, a.cC, left, right, up[0], dn[0], cen[0]);
            }
        } else {
            ldv<V>(uu + rn * nx + c0, udn);
            const double ul = uu[rw * nx + cl], ur = uu[rw * nx + cr];
            const double kc = -2.0 * a.kx - 2.0 * a.ky;
            if constexpr (V == 2) {
                o[0] = stencil_bu(a.kx, a.ky, a.gx, a.gy, kc, left, cen[1], up[0], dn[0], cen[0], ul, ucen[1], uup[0],
                                  udn[0]);
                o[1] = stencil_bu(a.kx, a.ky, a.gx, a.gy, kc, cen[0], right, up[1], dn[1], cen[1], ucen[0], ur, uup[1],
                                  udn[1]);
            } else {
                o[0] = stencil_bu(a.kx, a.ky, a.gx, a.gy, kc, left, right, up[0], dn[0], cen[0], ul, ur, uup[0], udn[0]);
            }
        }
        if (a.add != nullptr) {
            // s (A in + add): the right-hand side h (A u + S) of a linear step
            double sv[V];
            ldv<V>(a.add + rw * nx + c0, sv);
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = s * (o[i] + sv[i]);
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] *= s;
        }
        if (ok) {
            stv<V>(out + rw * nx + c0, o);
#pragma unroll
            for (int i = 0; i < V; ++i) acc += o[i] * o[i];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            if constexpr (OP == kOpDiffAdv3) up2[i] = up[i];
            up[i] = cen[i];
            cen[i] = dn[i];
            if constexpr (OP == kOpDiffAdv3) dn[i] = dn2[i];
            if constexpr (OP == kOpBurgersJ) {
                uup[i] = ucen[i];
                ucen[i] = udn[i];
            }
        }
    }
}

}  // namespace dev
}  // namespace lx
