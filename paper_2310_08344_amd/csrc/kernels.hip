// HIP kernels (gfx950) of the Leja phi-action library.
//
// One fused sweep per Leja iteration (Sec. 2.1, Eq. (2)):
//     y_{m+1} = ((A - c)/gamma - xi_m) y_m           (stencil, shifted centre)
//     p_k    += d^{(k)}_{m+1} y_{m+1}                (every unconverged output)
//     partial sums of |y_{m+1}|^2 and |p_k|^2         (norms of the stop rule)
// The last workgroup of a sweep to finish adds the per-workgroup partials in
// a fixed order, applies the stop rule of Sec. 2.2 and writes the loop state
// that the next sweep reads, so the loop never waits for the host.
//
// Memory layout: grids are row-major [ny][nx] (x fastest).  A thread owns
// `V` consecutive columns (one 16-byte FP64 load for V = 2) and marches down
// RY rows keeping the rows above, at and below in registers, so each row of
// y is fetched once per sweep; the x-neighbours of the pair come from the
// same cache lines through L1.  Workgroups are 2-D (tx lanes along x, ty
// thread-rows), 256 threads.  Consecutive workgroup ids go round-robin to
// the 8 XCDs; tiles are renumbered so that each XCD walks a contiguous band
// of rows and the halo rows of a tile were fetched by its own XCD shortly
// before.
#include <hip/hip_runtime.h>

#include "lx_device.h"

namespace lx {
namespace {

__device__ __forceinline__ int wrap(int r, int n) {
    if (r < 0) r += n;
    else if (r >= n) r -= n;
    if (r >= n) r %= n;      // only when a tile is taller than the grid
    return r;
}

__device__ __forceinline__ int tile_of_block(int b, int nb) {
    const int per = nb >> 3;
    if (per == 0 || b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int flat_tid() { return threadIdx.x + threadIdx.y * blockDim.x; }
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

// Sum NV values over the workgroup in a fixed order (butterfly within each
// 64-lane wavefront, then wavefronts in index order); the result is valid
// in thread 0 only.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NV][kBlockThreads / 64];
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
    if (tid == 0) {
        const int nw = (block_threads() + 63) >> 6;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[q][w];
            v[q] = s;
        }
    }
    __syncthreads();
}

// Publishes this workgroup's sums and reports whether it was the last of the
// grid to arrive; the last one then holds, in thread 0, the grid totals
// added in workgroup-index order (independent of arrival order).
template <int NV>
__device__ __forceinline__ bool grid_sum_last(double (&v)[NV], double* __restrict__ partials,
                                              unsigned* counter) {
    __shared__ int s_last;
    block_sum<NV>(v);
    const int tid = flat_tid();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[blockIdx.x * NV + q] = v[q];
        __threadfence();                                  // release the partials
        const unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();                                      // acquire the others' partials
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int b = tid; b < static_cast<int>(gridDim.x); b += block_threads()) {
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += __builtin_nontemporal_load(&partials[b * NV + q]);
    }
    block_sum<NV>(acc);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = acc[q];
    return true;
}

// ---------------------------------------------------------------------------
// Leja sweep
// ---------------------------------------------------------------------------

template <int OP, int K, int RY, int V, typename TI, typename TO, typename AT>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const int m, const int (&act)[K],
                                           double& sy, double (&sp)[K]) {
    const int nx = a.nx, ny = a.ny;
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int col = (tile_x * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) * V;
    const bool colok = col < nx;
    const int c0 = colok ? col : 0;
    const int cl = (c0 == 0) ? nx - 1 : c0 - 1;
    const int cr = (c0 + V >= nx) ? c0 + V - nx : c0 + V;
    const int row0 = tile_y * static_cast<int>(blockDim.y) * RY + static_cast<int>(threadIdx.y) * RY;

    const TI* __restrict__ yin;
    if constexpr (sizeof(TI) == sizeof(double)) {
        yin = (m == 0) ? reinterpret_cast<const TI*>(a.v) : static_cast<const TI*>(a.ybuf[(m - 1) & 1]);
    } else {
        yin = static_cast<const TI*>(a.ybuf[(m - 1) & 1]);
    }
    TO* __restrict__ yout = static_cast<TO*>(a.ybuf[m & 1]);

    const double xim = a.xi[m];
    double dn1[K], d0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dn1[k] = a.coef[k * a.ld + m + 1];
        d0[k] = a.coef[k * a.ld];
    }

    AT up[V], cen[V], dn[V];
    AT uup[V], ucen[V], udn[V];
    ldv<V>(yin + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, up);
    ldv<V>(yin + static_cast<long>(wrap(row0, ny)) * nx + c0, cen);
    if constexpr (OP == kOpBurgersJ) {
        if constexpr (sizeof(AT) == sizeof(double)) {
            ldv<V>(a.u + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
            ldv<V>(a.u + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
        } else {
            ldv<V>(a.u32 + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
            ldv<V>(a.u32 + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
        }
    }

#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int row = row0 + r;
        const bool ok = colok && row < ny;
        const long rw = wrap(row, ny);
        const long rn = wrap(row + 1, ny);
        ldv<V>(yin + rn * nx + c0, dn);
        const AT left = static_cast<AT>(yin[rw * nx + cl]);
        const AT right = static_cast<AT>(yin[rw * nx + cr]);
        AT o[V];
        if constexpr (OP == kOpDiffAdv) {
            const AT aE = static_cast<AT>(a.aE), aW = static_cast<AT>(a.aW);
            const AT aN = static_cast<AT>(a.aN), aS = static_cast<AT>(a.aS);
            const AT ac = static_cast<AT>(a.aC - xim);
            if constexpr (V == 2) {
                o[0] = aW * left + aE * cen[1] + aS * up[0] + aN * dn[0] + ac * cen[0];
                o[1] = aW * cen[0] + aE * right + aS * up[1] + aN * dn[1] + ac * cen[1];
            } else {
                o[0] = aW * left + aE * right + aS * up[0] + aN * dn[0] + ac * cen[0];
            }
        } else {
            const AT kx = static_cast<AT>(a.kx), ky = static_cast<AT>(a.ky);
            const AT gx = static_cast<AT>(a.gx), gy = static_cast<AT>(a.gy);
            const AT kc = static_cast<AT>(a.kC - xim);
            AT ul, ur;
            if constexpr (sizeof(AT) == sizeof(double)) {
                ldv<V>(a.u + rn * nx + c0, udn);
                ul = a.u[rw * nx + cl];
                ur = a.u[rw * nx + cr];
            } else {
                ldv<V>(a.u32 + rn * nx + c0, udn);
                ul = a.u32[rw * nx + cl];
                ur = a.u32[rw * nx + cr];
            }
            if constexpr (V == 2) {
                o[0] = kx * (cen[1] + left) + ky * (dn[0] + up[0]) - gx * (ucen[1] * cen[1] - ul * left) -
                       gy * (udn[0] * dn[0] - uup[0] * up[0]) + kc * cen[0];
                o[1] = kx * (right + cen[0]) + ky * (dn[1] + up[1]) - gx * (ur * right - ucen[0] * cen[0]) -
                       gy * (udn[1] * dn[1] - uup[1] * up[1]) + kc * cen[1];
            } else {
                o[0] = kx * (right + left) + ky * (dn[0] + up[0]) - gx * (ur * right - ul * left) -
                       gy * (udn[0] * dn[0] - uup[0] * up[0]) + kc * cen[0];
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
                // p_0 = d_0 y_0 (+ optional base); y_0 = v is the centre row
#pragma unroll
                for (int i = 0; i < V; ++i) pv[i] = d0[k] * static_cast<double>(cen[i]);
                if (a.base[k] != nullptr) {
                    double bv[V];
                    ldv<V>(a.base[k] + idx, bv);
#pragma unroll
                    for (int i = 0; i < V; ++i) pv[i] += bv[i];
                }
            } else {
                ldv<V>(a.p[k] + idx, pv);
            }
#pragma unroll
            for (int i = 0; i < V; ++i) pv[i] = fma(dn1[k], od[i], pv[i]);
            if (ok) {
                stv<V>(a.p[k] + idx, pv);
#pragma unroll
                for (int i = 0; i < V; ++i) sp[k] += pv[i] * pv[i];
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            up[i] = cen[i];
            cen[i] = dn[i];
            if constexpr (OP == kOpBurgersJ) {
                uup[i] = ucen[i];
                ucen[i] = udn[i];
            }
        }
    }
}

template <int OP, int K, int RY, int V, bool FP32>
__global__ __launch_bounds__(kBlockThreads) void leja_sweep(SweepArgs a) {
    LejaState* __restrict__ st = a.st;
    if (st->done) return;
    const int m = st->iter;
    int act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) act[k] = st->active[k];
    double sy = 0.0, sp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sp[k] = 0.0;
    int wrote32 = 0;
    if constexpr (FP32) {
        const int in32 = st->in32, out32 = st->out32;
        wrote32 = out32;
        if (in32) {
            sweep_tile<OP, K, RY, V, float, float, float>(a, m, act, sy, sp);
        } else if (out32) {
            sweep_tile<OP, K, RY, V, double, float, double>(a, m, act, sy, sp);
        } else {
            sweep_tile<OP, K, RY, V, double, double, double>(a, m, act, sy, sp);
        }
    } else {
        sweep_tile<OP, K, RY, V, double, double, double>(a, m, act, sy, sp);
    }

    double v[1 + K];
    v[0] = sy;
#pragma unroll
    for (int k = 0; k < K; ++k) v[1 + k] = sp[k];
    if (!grid_sum_last<1 + K>(v, a.partials, &st->arrive)) return;
    if (flat_tid() != 0) return;

    // stop rule (Sec. 2.2): |d_{m+1}| ||y_{m+1}|| <= rtol ||p|| + atol, rms norms
    const double ynorm = sqrt(v[0]) * a.inv_sqrtN;
    bool nonfinite = !isfinite(ynorm);
    bool any_active = false, all_small = true;
    const double rtol = st->rtol, atol = st->atol, sw = st->fp32_switch;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!act[k]) continue;
        const double pn = sqrt(v[1 + k]) * a.inv_sqrtN;
        const double e = fabs(a.coef[k * a.ld + m + 1]) * ynorm;
        const double thr = rtol * pn + atol;
        st->err[k] = e;
        st->pnorm[k] = pn;
        if (!isfinite(pn) || !isfinite(e)) {
            nonfinite = true;
            st->active[k] = 0;
            st->iters[k] = m + 1;
        } else if (e <= thr) {
            st->active[k] = 0;
            st->iters[k] = m + 1;
        } else {
            any_active = true;
            if (!(e <= sw * thr)) all_small = false;
        }
    }
    st->ynorm = ynorm;
    st->iter = m + 1;
    st->in32 = wrote32;
    st->n_fp32 += wrote32;
    if (FP32 && !wrote32 && any_active && all_small && sw >= 0.0) st->out32 = 1;
    if (nonfinite) {
        st->status = 4;  // LX_ENONFINITE
        st->done = 1;
    } else if (!any_active) {
        st->status = 0;
        st->done = 1;
    } else if (m + 1 >= st->max_iters) {
        st->status = 3;  // LX_ENOTCONV
        st->done = 1;
    }
    st->arrive = 0u;
    __threadfence();
}

// ---------------------------------------------------------------------------
// power iteration sweep: w_out = (A w_in) / ||w_in||, partial sums of w_out^2
// ---------------------------------------------------------------------------

template <int OP, int RY, int V>
__global__ __launch_bounds__(kBlockThreads) void power_sweep(PowerArgs a) {
    LejaState* __restrict__ st = a.st;
    const double s = st->scale;
    const int nx = a.nx, ny = a.ny;
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int col = (tile_x * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) * V;
    const bool colok = col < nx;
    const int c0 = colok ? col : 0;
    const int cl = (c0 == 0) ? nx - 1 : c0 - 1;
    const int cr = (c0 + V >= nx) ? c0 + V - nx : c0 + V;
    const int row0 = tile_y * static_cast<int>(blockDim.y) * RY + static_cast<int>(threadIdx.y) * RY;
    const double* __restrict__ in = a.in;

    double up[V], cen[V], dn[V], uup[V], ucen[V], udn[V];
    ldv<V>(in + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, up);
    ldv<V>(in + static_cast<long>(wrap(row0, ny)) * nx + c0, cen);
    if constexpr (OP == kOpBurgersJ) {
        ldv<V>(a.u + static_cast<long>(wrap(row0 - 1, ny)) * nx + c0, uup);
        ldv<V>(a.u + static_cast<long>(wrap(row0, ny)) * nx + c0, ucen);
    }
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int row = row0 + r;
        const bool ok = colok && row < ny;
        const long rw = wrap(row, ny);
        const long rn = wrap(row + 1, ny);
        ldv<V>(in + rn * nx + c0, dn);
        const double left = in[rw * nx + cl], right = in[rw * nx + cr];
        double o[V];
        if constexpr (OP == kOpDiffAdv) {
            if constexpr (V == 2) {
                o[0] = a.cW * left + a.cE * cen[1] + a.cS * up[0] + a.cN * dn[0] + a.cC * cen[0];
                o[1] = a.cW * cen[0] + a.cE * right + a.cS * up[1] + a.cN * dn[1] + a.cC * cen[1];
            } else {
                o[0] = a.cW * left + a.cE * right + a.cS * up[0] + a.cN * dn[0] + a.cC * cen[0];
            }
        } else {
            ldv<V>(a.u + rn * nx + c0, udn);
            const double ul = a.u[rw * nx + cl], ur = a.u[rw * nx + cr];
            const double kc = -2.0 * a.kx - 2.0 * a.ky;
            if constexpr (V == 2) {
                o[0] = a.kx * (cen[1] + left) + a.ky * (dn[0] + up[0]) - a.gx * (ucen[1] * cen[1] - ul * left) -
                       a.gy * (udn[0] * dn[0] - uup[0] * up[0]) + kc * cen[0];
                o[1] = a.kx * (right + cen[0]) + a.ky * (dn[1] + up[1]) - a.gx * (ur * right - ucen[0] * cen[0]) -
                       a.gy * (udn[1] * dn[1] - uup[1] * up[1]) + kc * cen[1];
            } else {
                o[0] = a.kx * (right + left) + a.ky * (dn[0] + up[0]) - a.gx * (ur * right - ul * left) -
                       a.gy * (udn[0] * dn[0] - uup[0] * up[0]) + kc * cen[0];
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] *= s;
        if (ok) {
            stv<V>(a.out + rw * nx + c0, o);
#pragma unroll
            for (int i = 0; i < V; ++i) acc += o[i] * o[i];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            up[i] = cen[i];
            cen[i] = dn[i];
            if constexpr (OP == kOpBurgersJ) {
                uup[i] = ucen[i];
                ucen[i] = udn[i];
            }
        }
    }
    double v[1] = {acc};
    if (!grid_sum_last<1>(v, a.partials, &st->arrive)) return;
    if (flat_tid() != 0) return;
    const double nrm = sqrt(v[0]);
    st->rho = nrm;
    st->scale = 1.0 / nrm;
    st->iter += 1;
    if (!isfinite(nrm) || nrm == 0.0) st->status = 4;
    st->arrive = 0u;
    __threadfence();
}

// ||x|| of the start vector: st->scale = 1/||x||
__global__ __launch_bounds__(kBlockThreads) void norm_kernel(const double* __restrict__ x, long n,
                                                             double* partials, LejaState* st) {
    double acc = 0.0;
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        const double t = x[i];
        acc += t * t;
    }
    double v[1] = {acc};
    if (!grid_sum_last<1>(v, partials, &st->arrive)) return;
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(v[0]);
    st->scale = 1.0 / nrm;
    if (!isfinite(nrm) || nrm == 0.0) st->status = 4;
    st->arrive = 0u;
    __threadfence();
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014): state_i = seed + (i+1) *
// 0x9e3779b97f4a7c15, then the published output mix; value in [-1, 1)
__global__ void fill_splitmix_kernel(double* __restrict__ x, long n, unsigned long long seed) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        unsigned long long z = seed + static_cast<unsigned long long>(i + 1) * 0x9e3779b97f4a7c15ULL;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        x[i] = static_cast<double>(z >> 11) * 0x1.0p-52 - 1.0;
    }
}

__global__ void to_fp32_kernel(const double* __restrict__ x, float* __restrict__ y, long n) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        y[i] = static_cast<float>(x[i]);
    }
}

// Burgers right-hand side pieces (one point per thread, used once per step)
__device__ __forceinline__ double burgers_F_at(const double* __restrict__ u, int i, int j, int nx, int ny,
                                               double nu, double dx, double dy) {
    const int ie = (i + 1 == nx) ? 0 : i + 1, iw = (i == 0) ? nx - 1 : i - 1;
    const int jn = (j + 1 == ny) ? 0 : j + 1, js = (j == 0) ? ny - 1 : j - 1;
    const double c = u[static_cast<long>(j) * nx + i];
    const double e = u[static_cast<long>(j) * nx + ie], w = u[static_cast<long>(j) * nx + iw];
    const double nn = u[static_cast<long>(jn) * nx + i], s = u[static_cast<long>(js) * nx + i];
    const double lap = (e - 2.0 * c + w) / (dx * dx) + (nn - 2.0 * c + s) / (dy * dy);
    const double div = (e * e - w * w) / (2.0 * dx) + (nn * nn - s * s) / (2.0 * dy);
    return nu * lap - 0.5 * div;
}

__global__ void burgers_hF_kernel(const double* __restrict__ u, double* __restrict__ out, int nx, int ny,
                                  double nu, double dx, double dy, double h) {
    const long n = static_cast<long>(nx) * ny;
    for (long t = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(t % nx), j = static_cast<int>(t / nx);
        out[t] = h * burgers_F_at(u, i, j, nx, ny, nu, dx, dy);
    }
}

// R = h [N(U2) - N(u)] with N(w) = F(w) - J(u) w, i.e.
// h [F(U2) - F(u) - J(u)(U2 - u)]
__global__ void burgers_remainder_kernel(const double* __restrict__ u, const double* __restrict__ U2,
                                         double* __restrict__ out, int nx, int ny, double nu, double dx,
                                         double dy, double h) {
    const long n = static_cast<long>(nx) * ny;
    for (long t = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(t % nx), j = static_cast<int>(t / nx);
        const int ie = (i + 1 == nx) ? 0 : i + 1, iw = (i == 0) ? nx - 1 : i - 1;
        const int jn = (j + 1 == ny) ? 0 : j + 1, js = (j == 0) ? ny - 1 : j - 1;
        const long ce = static_cast<long>(j) * nx + ie, cw = static_cast<long>(j) * nx + iw;
        const long cn = static_cast<long>(jn) * nx + i, cs = static_cast<long>(js) * nx + i;
        const double ae = U2[ce] - u[ce], aw = U2[cw] - u[cw], an = U2[cn] - u[cn], as = U2[cs] - u[cs];
        const double ac = U2[t] - u[t];
        const double lap = (ae - 2.0 * ac + aw) / (dx * dx) + (an - 2.0 * ac + as) / (dy * dy);
        const double Ja = nu * lap - ((u[ce] * ae - u[cw] * aw) / (2.0 * dx) + (u[cn] * an - u[cs] * as) / (2.0 * dy));
        const double FU2 = burgers_F_at(U2, i, j, nx, ny, nu, dx, dy);
        const double Fu = burgers_F_at(u, i, j, nx, ny, nu, dx, dy);
        out[t] = h * (FU2 - Fu - Ja);
    }
}

// ---------------------------------------------------------------------------
// launch dispatch
// ---------------------------------------------------------------------------

template <int OP, int K, int RY, int V>
hipError_t launch_sweep_t(bool fp32, const Tile& t, const SweepArgs& a, hipStream_t s) {
    const dim3 block(t.tx, t.ty);
    const dim3 grid(a.tiles_x * a.tiles_y);
    if (fp32) {
        hipLaunchKernelGGL((leja_sweep<OP, K, RY, V, true>), grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((leja_sweep<OP, K, RY, V, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int OP, int K, int RY>
hipError_t launch_sweep_v(bool fp32, const Tile& t, const SweepArgs& a, hipStream_t s) {
    return t.vec == 2 ? launch_sweep_t<OP, K, RY, 2>(fp32, t, a, s) : launch_sweep_t<OP, K, RY, 1>(fp32, t, a, s);
}

template <int OP, int K>
hipError_t launch_sweep_r(bool fp32, const Tile& t, const SweepArgs& a, hipStream_t s) {
    switch (t.ry) {
        case 1: return launch_sweep_v<OP, K, 1>(fp32, t, a, s);
        case 2: return launch_sweep_v<OP, K, 2>(fp32, t, a, s);
        case 4: return launch_sweep_v<OP, K, 4>(fp32, t, a, s);
        case 8: return launch_sweep_v<OP, K, 8>(fp32, t, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int OP>
hipError_t launch_sweep_k(int K, bool fp32, const Tile& t, const SweepArgs& a, hipStream_t s) {
    switch (K) {
        case 1: return launch_sweep_r<OP, 1>(fp32, t, a, s);
        case 2: return launch_sweep_r<OP, 2>(fp32, t, a, s);
        case 3: return launch_sweep_r<OP, 3>(fp32, t, a, s);
        case 4: return launch_sweep_r<OP, 4>(fp32, t, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int OP, int RY, int V>
hipError_t launch_power_t(const Tile& t, const PowerArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((power_sweep<OP, RY, V>), dim3(a.tiles_x * a.tiles_y), dim3(t.tx, t.ty), 0, s, a);
    return hipGetLastError();
}

template <int OP, int RY>
hipError_t launch_power_v(const Tile& t, const PowerArgs& a, hipStream_t s) {
    return t.vec == 2 ? launch_power_t<OP, RY, 2>(t, a, s) : launch_power_t<OP, RY, 1>(t, a, s);
}

template <int OP>
hipError_t launch_power_r(const Tile& t, const PowerArgs& a, hipStream_t s) {
    switch (t.ry) {
        case 1: return launch_power_v<OP, 1>(t, a, s);
        case 2: return launch_power_v<OP, 2>(t, a, s);
        case 4: return launch_power_v<OP, 4>(t, a, s);
        case 8: return launch_power_v<OP, 8>(t, a, s);
        default: return hipErrorInvalidValue;
    }
}

int flat_blocks(long n) {
    long b = (n + kBlockThreads - 1) / kBlockThreads;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

}  // namespace

int num_blocks(const Tile& t, int nx, int ny) {
    const int tx = (nx + t.cols() - 1) / t.cols();
    const int ty = (ny + t.rows() - 1) / t.rows();
    return tx * ty;
}

int norm_blocks(long n) { return flat_blocks(n); }

hipError_t launch_leja_sweep(int op, int K, bool fp32_capable, const Tile& t, const SweepArgs& a,
                             hipStream_t s) {
    if (t.tx * t.ty != kBlockThreads) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_sweep_k<kOpDiffAdv>(K, fp32_capable, t, a, s);
    if (op == kOpBurgersJ) return launch_sweep_k<kOpBurgersJ>(K, fp32_capable, t, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_power_sweep(int op, const Tile& t, const PowerArgs& a, hipStream_t s) {
    if (t.tx * t.ty != kBlockThreads) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_power_r<kOpDiffAdv>(t, a, s);
    if (op == kOpBurgersJ) return launch_power_r<kOpBurgersJ>(t, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_norm(const double* x, long n, double* partials, LejaState* st, hipStream_t s) {
    hipLaunchKernelGGL(norm_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, x, n, partials, st);
    return hipGetLastError();
}

hipError_t launch_fill_splitmix(double* x, long n, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(fill_splitmix_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_to_fp32(const double* x, float* y, long n, hipStream_t s) {
    hipLaunchKernelGGL(to_fp32_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_burgers_hF(const double* u, double* out, int nx, int ny, double nu, double dx, double dy,
                             double h, hipStream_t s) {
    hipLaunchKernelGGL(burgers_hF_kernel, dim3(flat_blocks(static_cast<long>(nx) * ny)), dim3(kBlockThreads), 0,
                       s, u, out, nx, ny, nu, dx, dy, h);
    return hipGetLastError();
}

hipError_t launch_burgers_remainder(const double* u, const double* U2, double* out, int nx, int ny, double nu,
                                    double dx, double dy, double h, hipStream_t s) {
    hipLaunchKernelGGL(burgers_remainder_kernel, dim3(flat_blocks(static_cast<long>(nx) * ny)),
                       dim3(kBlockThreads), 0, s, u, U2, out, nx, ny, nu, dx, dy, h);
    return hipGetLastError();
}

}  // namespace lx
