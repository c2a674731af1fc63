// HIP kernels (gfx950) of the Leja phi-action library.
//
// One fused sweep per Leja iteration (Sec. 2.1, Eq. (2)):
//     y_{m+1} = ((A - c)/gamma - xi_m) y_m           (stencil, shifted centre)
//     p_k    += d^{(k)}_{m+1} y_{m+1}                (every unconverged output)
//     partial sums of |y_{m+1}|^2 and |p_k|^2         (norms of the stop rule)
// Sweeps never synchronise their workgroups.  Each workgroup writes its
// partial sums with plain stores; at the start of the next sweep every
// workgroup adds all of them in the same fixed order and so takes the same
// stop decision (Sec. 2.2) on its own.  The kernel boundary is the only
// grid-wide barrier: on MI355X the L2 caches of the 8 XCDs are not coherent
// with each other, and a device-scope release inside a sweep (needed by a
// last-workgroup reduction) costs an L2 write-back per workgroup.
//
// Memory layout: grids are row-major [ny][nx] (x fastest).  A thread owns
// `V` consecutive columns (one 16-byte FP64 load for V = 2) and marches down
// RY rows keeping the rows above, at and below in registers, so each row of
// y is fetched once per tile; the x-neighbours of the pair come from the
// same cache lines through L1.  Workgroups are 2-D (tx lanes along x, ty
// thread-rows), 256 threads, and loop over tiles.  Consecutive workgroup
// ids go round-robin to the 8 XCDs; the tiles are split into 8 contiguous
// bands, one per XCD, so that a tile's halo rows were fetched by its own
// XCD shortly before.
#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"

namespace lx {
namespace {

using namespace dev;

template <int OP, int K, int RY, int V, bool FP32>
__global__ __launch_bounds__(kBlockThreads) void leja_sweep(SweepArgs a, const int m) {
    LoopCtl* __restrict__ ctl = a.ctl;
    if (loop_ended(ctl)) return;
    constexpr int NV = 1 + K;
    __shared__ SweepState s_cur;
    const int tid = flat_tid();
    if (m == 0) {
        if (tid == 0) s_cur = ctl->slot[0];
    } else {
        double tot[NV];
        sum_partials<NV>(a.partials + static_cast<long>((m - 1) & 1) * a.nb * NV, a.nb, tot);
        if (tid == 0) {
            const SweepState nxt = decide<K, FP32>(a, *ctl, ctl->slot[(m - 1) & 1], m, tot);
            s_cur = nxt;
            if (blockIdx.x == 0) {
                ctl->slot[m & 1] = nxt;
                if (nxt.done) publish_final(ctl, a.pub, nxt);
            }
        }
    }
    __syncthreads();
    if (s_cur.done) return;

    int act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) act[k] = s_cur.active[k];
    double sy = 0.0, sp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sp[k] = 0.0;
    const int T = a.tiles_x * a.tiles_y;
    if constexpr (FP32) {
        if (s_cur.in32) {
            for_each_tile(T, a.nb, [&](int t) { sweep_tile<OP, K, RY, V, float, float, float>(a, m, act, sy, sp, t); });
        } else if (s_cur.out32) {
            for_each_tile(T, a.nb,
                          [&](int t) { sweep_tile<OP, K, RY, V, double, float, double>(a, m, act, sy, sp, t); });
        } else {
            for_each_tile(T, a.nb,
                          [&](int t) { sweep_tile<OP, K, RY, V, double, double, double>(a, m, act, sy, sp, t); });
        }
    } else {
        for_each_tile(T, a.nb,
                      [&](int t) { sweep_tile<OP, K, RY, V, double, double, double>(a, m, act, sy, sp, t); });
    }
    double v[NV];
    v[0] = sy;
#pragma unroll
    for (int k = 0; k < K; ++k) v[1 + k] = sp[k];
    block_sum<NV>(v);
    if (tid == 0) {
        double* __restrict__ P = a.partials + static_cast<long>(m & 1) * a.nb * NV + blockIdx.x * NV;
#pragma unroll
        for (int q = 0; q < NV; ++q) P[q] = v[q];
    }
}

template <int OP, int RY, int V>
__global__ __launch_bounds__(kBlockThreads) void power_sweep(PowerArgs a, const int k) {
    double tot[1];
    sum_partials<1>(a.partials + static_cast<long>((k - 1) & 1) * a.nb, a.nb, tot);
    const double s = 1.0 / sqrt(tot[0]);
    double acc = 0.0;
    for_each_tile(a.tiles_x * a.tiles_y, a.nb, [&](int t) { power_tile<OP, RY, V>(a, s, acc, t); });
    double v[1] = {acc};
    block_sum<1>(v);
    if (flat_tid() == 0) a.partials[static_cast<long>(k & 1) * a.nb + blockIdx.x] = v[0];
}

// h (A u + S), tiled like the power sweep (the sums of squares are unused)
template <int OP, int RY, int V>
__global__ __launch_bounds__(kBlockThreads) void rhs_sweep(PowerArgs a, const double h) {
    double acc = 0.0;
    for_each_tile(a.tiles_x * a.tiles_y, a.nb, [&](int t) { power_tile<OP, RY, V>(a, h, acc, t); });
}

// partial sums of |x|^2 of the start vector into partials[1][*]; 16-byte
// loads, four in flight per thread, when x is 16-byte aligned
__global__ __launch_bounds__(kBlockThreads) void power_norm_kernel(const double* __restrict__ x, long n,
                                                                   double* __restrict__ partials) {
    const long tid = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
    const long G = static_cast<long>(gridDim.x) * blockDim.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);
        const long n2 = n / 2;
        long i = tid;
        for (; i + 3 * G < n2; i += 4 * G) {
            double2 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = x2[i + q * G];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += v[q].x * v[q].x + v[q].y * v[q].y;
        }
        for (; i < n2; i += G) acc[0] += x2[i].x * x2[i].x + x2[i].y * x2[i].y;
        if ((n & 1) && tid == 0) acc[1] += x[n - 1] * x[n - 1];
    } else {
        for (long i = tid; i < n; i += G) acc[0] += x[i] * x[i];
    }
    double v[1] = {(acc[0] + acc[1]) + (acc[2] + acc[3])};
    block_sum<1>(v);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = v[0];
}

// rho = ||w_iters|| from the last sweep's partial sums
__global__ __launch_bounds__(kBlockThreads) void power_final_kernel(int nb, const double* __restrict__ P,
                                                                    LoopCtl* ctl) {
    double tot[1];
    sum_partials<1>(P, nb, tot);
    if (threadIdx.x == 0) ctl->rho = sqrt(tot[0]);
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

// R = h [N(u + a) - N(u)] with N(w) = F(w) - J(u) w, i.e.
// h [F(w) - F(u) - J(u) a] for the stage w = u + a (formed here, as the
// stage vector of the integrator)
__global__ void burgers_remainder_kernel(const double* __restrict__ u, const double* __restrict__ a,
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
        const double ac = a[t], ae = a[ce], aw = a[cw], an = a[cn], as = a[cs];
        const double wc = u[t] + ac, we = u[ce] + ae, ww = u[cw] + aw, wn = u[cn] + an, ws = u[cs] + as;
        const double lapw = (we - 2.0 * wc + ww) / (dx * dx) + (wn - 2.0 * wc + ws) / (dy * dy);
        const double Fw = nu * lapw - 0.5 * ((we * we - ww * ww) / (2.0 * dx) + (wn * wn - ws * ws) / (2.0 * dy));
        const double lapa = (ae - 2.0 * ac + aw) / (dx * dx) + (an - 2.0 * ac + as) / (dy * dy);
        const double Ja = nu * lapa - ((u[ce] * ae - u[cw] * aw) / (2.0 * dx) + (u[cn] * an - u[cs] * as) / (2.0 * dy));
        const double Fu = burgers_F_at(u, i, j, nx, ny, nu, dx, dy);
        out[t] = h * (Fw - Fu - Ja);
    }
}

// out = b base + sum_i a_i x_i, base optional: the substep updates of
// phi-function time stepping
__global__ void lincomb_kernel(double* __restrict__ out, const double* __restrict__ base, double b, LinComb t,
                               long n) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        double r = (base != nullptr) ? b * base[i] : 0.0;
        for (int k = 0; k < t.n_terms; ++k) r = fma(t.a[k], t.x[k][i], r);
        out[i] = r;
    }
}

// out = (x + y) + z, z optional (the stages of the integrators)
__global__ void combine_kernel(const double* __restrict__ x, const double* __restrict__ y,
                               const double* __restrict__ z, double* __restrict__ out, long n) {
    for (long t = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<long>(gridDim.x) * blockDim.x) {
        const double s = x[t] + y[t];
        out[t] = (z != nullptr) ? s + z[t] : s;
    }
}

// ---------------------------------------------------------------------------
// streaming probes: the practical-bandwidth calibration of Sec. 3 (device
// copy and z = a x + b y)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlockThreads) void copy_kernel(const double2* __restrict__ x,
                                                             double2* __restrict__ y, long n2) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n2;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        y[i] = x[i];
    }
}

__global__ __launch_bounds__(kBlockThreads) void axpby_kernel(double a, const double2* __restrict__ x, double b,
                                                              const double2* __restrict__ y,
                                                              double2* __restrict__ z, long n2) {
    for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n2;
         i += static_cast<long>(gridDim.x) * blockDim.x) {
        const double2 xv = x[i], yv = y[i];
        double2 r;
        r.x = a * xv.x + b * yv.x;
        r.y = a * xv.y + b * yv.y;
        z[i] = r;
    }
}

// ---------------------------------------------------------------------------
// launch dispatch
// ---------------------------------------------------------------------------

template <int OP, int K, int RY, int V>
hipError_t launch_sweep_t(bool fp32, const Tile& t, const SweepArgs& a, int m, hipStream_t s) {
    const dim3 block(t.tx, t.ty);
    const dim3 grid(a.nb);
    if (fp32) {
        hipLaunchKernelGGL((leja_sweep<OP, K, RY, V, true>), grid, block, 0, s, a, m);
    } else {
        hipLaunchKernelGGL((leja_sweep<OP, K, RY, V, false>), grid, block, 0, s, a, m);
    }
    return hipGetLastError();
}

template <int OP, int K, int RY>
hipError_t launch_sweep_v(bool fp32, const Tile& t, const SweepArgs& a, int m, hipStream_t s) {
    return t.vec == 2 ? launch_sweep_t<OP, K, RY, 2>(fp32, t, a, m, s) : launch_sweep_t<OP, K, RY, 1>(fp32, t, a, m, s);
}

template <int OP, int K>
hipError_t launch_sweep_r(bool fp32, const Tile& t, const SweepArgs& a, int m, hipStream_t s) {
    switch (t.ry) {
        case 1: return launch_sweep_v<OP, K, 1>(fp32, t, a, m, s);
        case 2: return launch_sweep_v<OP, K, 2>(fp32, t, a, m, s);
        case 4: return launch_sweep_v<OP, K, 4>(fp32, t, a, m, s);
        case 8: return launch_sweep_v<OP, K, 8>(fp32, t, a, m, s);
        default: return hipErrorInvalidValue;
    }
}

template <int OP>
hipError_t launch_sweep_k(int K, bool fp32, const Tile& t, const SweepArgs& a, int m, hipStream_t s) {
    switch (K) {
        case 1: return launch_sweep_r<OP, 1>(fp32, t, a, m, s);
        case 2: return launch_sweep_r<OP, 2>(fp32, t, a, m, s);
        case 3: return launch_sweep_r<OP, 3>(fp32, t, a, m, s);
        case 4: return launch_sweep_r<OP, 4>(fp32, t, a, m, s);
        default: return hipErrorInvalidValue;
    }
}

template <int OP, int RY, int V>
hipError_t launch_power_t(const Tile& t, const PowerArgs& a, int k, hipStream_t s) {
    hipLaunchKernelGGL((power_sweep<OP, RY, V>), dim3(a.nb), dim3(t.tx, t.ty), 0, s, a, k);
    return hipGetLastError();
}

template <int OP, int RY>
hipError_t launch_power_v(const Tile& t, const PowerArgs& a, int k, hipStream_t s) {
    return t.vec == 2 ? launch_power_t<OP, RY, 2>(t, a, k, s) : launch_power_t<OP, RY, 1>(t, a, k, s);
}

template <int OP>
hipError_t launch_power_r(const Tile& t, const PowerArgs& a, int k, hipStream_t s) {
    switch (t.ry) {
        case 1: return launch_power_v<OP, 1>(t, a, k, s);
        case 2: return launch_power_v<OP, 2>(t, a, k, s);
        case 4: return launch_power_v<OP, 4>(t, a, k, s);
        case 8: return launch_power_v<OP, 8>(t, a, k, s);
        default: return hipErrorInvalidValue;
    }
}

template <int OP, int RY>
hipError_t launch_rhs_v(const Tile& t, const PowerArgs& a, double h, hipStream_t s) {
    if (t.vec == 2) hipLaunchKernelGGL((rhs_sweep<OP, RY, 2>), dim3(a.nb), dim3(t.tx, t.ty), 0, s, a, h);
    else hipLaunchKernelGGL((rhs_sweep<OP, RY, 1>), dim3(a.nb), dim3(t.tx, t.ty), 0, s, a, h);
    return hipGetLastError();
}

template <int OP>
hipError_t launch_rhs_r(const Tile& t, const PowerArgs& a, double h, hipStream_t s) {
    switch (t.ry) {
        case 1: return launch_rhs_v<OP, 1>(t, a, h, s);
        case 2: return launch_rhs_v<OP, 2>(t, a, h, s);
        case 4: return launch_rhs_v<OP, 4>(t, a, h, s);
        case 8: return launch_rhs_v<OP, 8>(t, a, h, s);
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

hipError_t launch_leja_sweep(int op, int K, bool fp32_capable, const Tile& t, const SweepArgs& a, int m,
                             hipStream_t s) {
    if (t.tx * t.ty != kBlockThreads || a.nb < 1) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_sweep_k<kOpDiffAdv>(K, fp32_capable, t, a, m, s);
    if (op == kOpBurgersJ) return launch_sweep_k<kOpBurgersJ>(K, fp32_capable, t, a, m, s);
    if (op == kOpDiffAdv3) return launch_sweep_k<kOpDiffAdv3>(K, fp32_capable, t, a, m, s);
    return hipErrorInvalidValue;
}

hipError_t launch_power_sweep(int op, const Tile& t, const PowerArgs& a, int k, hipStream_t s) {
    if (t.tx * t.ty != kBlockThreads || a.nb < 1) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_power_r<kOpDiffAdv>(t, a, k, s);
    if (op == kOpBurgersJ) return launch_power_r<kOpBurgersJ>(t, a, k, s);
    if (op == kOpDiffAdv3) return launch_power_r<kOpDiffAdv3>(t, a, k, s);
    return hipErrorInvalidValue;
}

hipError_t launch_rhs_sweep(int op, const Tile& t, const PowerArgs& a, double h, hipStream_t s) {
    if (t.tx * t.ty != kBlockThreads || a.nb < 1) return hipErrorInvalidValue;
    if (op == kOpDiffAdv) return launch_rhs_r<kOpDiffAdv>(t, a, h, s);
    if (op == kOpDiffAdv3) return launch_rhs_r<kOpDiffAdv3>(t, a, h, s);
    return hipErrorInvalidValue;
}

hipError_t launch_power_norm(const double* x, long n, int nb, double* partials, hipStream_t s) {
    if (nb < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(power_norm_kernel, dim3(nb), dim3(kBlockThreads), 0, s, x, n, partials);
    return hipGetLastError();
}

hipError_t launch_power_final(int nb, const double* partials, LoopCtl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(power_final_kernel, dim3(1), dim3(kBlockThreads), 0, s, nb, partials, ctl);
    return hipGetLastError();
}

hipError_t launch_fill_splitmix(double* x, long n, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(fill_splitmix_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_probe(int kind, const double* x, const double* y, double* z, long n, hipStream_t s) {
    const long n2 = n / 2;
    long blocks = (n2 + kBlockThreads - 1) / kBlockThreads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (kind == 0) {
        hipLaunchKernelGGL(copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlockThreads), 0, s,
                           reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(z), n2);
    } else {
        hipLaunchKernelGGL(axpby_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlockThreads), 0, s, 1.5,
                           reinterpret_cast<const double2*>(x), -0.5, reinterpret_cast<const double2*>(y),
                           reinterpret_cast<double2*>(z), n2);
    }
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

hipError_t launch_burgers_remainder(const double* u, const double* a, double* out, int nx, int ny, double nu,
                                    double dx, double dy, double h, hipStream_t s) {
    hipLaunchKernelGGL(burgers_remainder_kernel, dim3(flat_blocks(static_cast<long>(nx) * ny)),
                       dim3(kBlockThreads), 0, s, u, a, out, nx, ny, nu, dx, dy, h);
    return hipGetLastError();
}

hipError_t launch_lincomb(double* out, const double* base, double b, const LinComb& t, long n, hipStream_t s) {
    if (t.n_terms < 0 || t.n_terms > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lincomb_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, out, base, b, t, n);
    return hipGetLastError();
}

hipError_t launch_combine(const double* x, const double* y, const double* z, double* out, long n, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(flat_blocks(n)), dim3(kBlockThreads), 0, s, x, y, z, out, n);
    return hipGetLastError();
}

}  // namespace lx
