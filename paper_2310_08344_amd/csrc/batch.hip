// Batched kernels (gfx950): many independent phi-action problems of uneven
// size advance together, one launch per sweep for the whole batch.
//
// Every workgroup serves one instance (block_inst[blockIdx.x]) and loops
// over that instance's tiles.  Each instance has its own loop control, its
// own parity-buffered partial sums and its own stop decision, taken by all
// of its workgroups from the same partials in the same order, exactly as in
// the single-grid sweep (Sec. 2.1, Eq. (2); stop rule of Sec. 2.2).
// Instances that have finished return at entry, so the batch costs what
// its unfinished instances move.  The spectral bounds (power iteration,
// Listing 7) and the Newton coefficients are computed on the device as
// well, so a whole batch runs without a host round trip per instance.
#include <hip/hip_runtime.h>

#include "dd_math.h"
#include "lx_device.h"
#include "stencil_coeffs.h"
#include "sweep_device.h"

namespace lx {
namespace {

using namespace dev;

constexpr int kCoefThreads = 64;
constexpr int kMaxCoef = 1008;   // coefficients per instance: up to max_iters + 1 + the window depth

struct Who {
    int i;   // instance
    int j;   // workgroup index within the instance
};

__device__ __forceinline__ Who who(const BatchInst* insts, const int* block_inst) {
    const int i = block_inst[blockIdx.x];
    return {i, static_cast<int>(blockIdx.x) - insts[i].wg_begin};
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014) of the instance's seed
// (its index) at position t, mapped to [-1, 1)
__device__ __forceinline__ double splitmix_unit(unsigned long long seed, long t) {
    unsigned long long z = seed + static_cast<unsigned long long>(t + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return static_cast<double>(z >> 11) * 0x1.0p-52 - 1.0;
}

__global__ __launch_bounds__(kBlockThreads) void batch_fill_x0_kernel(BatchInst* insts, const int* block_inst) {
    const Who w = who(insts, block_inst);
    const BatchInst& I = insts[w.i];
    if (I.has_x0) return;
    const long n = static_cast<long>(I.nx) * I.ny;
    double* __restrict__ x = gptr(I.y[1]);
    for (long t = static_cast<long>(w.j) * kBlockThreads + flat_tid(); t < n;
         t += static_cast<long>(I.nb) * kBlockThreads) {
        x[t] = splitmix_unit(static_cast<unsigned long long>(w.i), t);
    }
}

__global__ __launch_bounds__(kBlockThreads) void batch_power_norm_kernel(const BatchInst* insts,
                                                                         const int* block_inst,
                                                                         double* partials) {
    const Who w = who(insts, block_inst);
    const BatchInst& I = insts[w.i];
    const double* __restrict__ x = gptr(I.has_x0 ? I.x0 : I.y[1]);
    const long n = static_cast<long>(I.nx) * I.ny;
    double acc = 0.0;
    for (long t = static_cast<long>(w.j) * kBlockThreads + flat_tid(); t < n;
         t += static_cast<long>(I.nb) * kBlockThreads) {
        const double q = x[t];
        acc += q * q;
    }
    double v[1] = {acc};
    block_sum<1>(v);
    if (flat_tid() == 0) partials[I.part_off + I.nb + w.j] = v[0];   // slot 1
}

__device__ __forceinline__ void power_coeffs(const BatchInst& I, PowerArgs& a) {
    if (I.kind == kOpDiffAdv) {
        a.cE = I.pw[0];
        a.cW = I.pw[1];
        a.cN = I.pw[2];
        a.cS = I.pw[3];
        a.cC = I.pw[4];
    } else {
        a.kx = I.pw[0];
        a.ky = I.pw[1];
        a.gx = I.pw[2];
        a.gy = I.pw[3];
    }
}

__global__ __launch_bounds__(kBlockThreads) void batch_power_sweep_kernel(const BatchInst* insts,
                                                                          const int* block_inst,
                                                                          double* partials, const int k) {
    const Who w = who(insts, block_inst);
    const BatchInst& I = insts[w.i];
    double* __restrict__ P = partials + I.part_off;
    double tot[1];
    sum_partials<1>(P + static_cast<long>((k - 1) & 1) * I.nb, I.nb, tot);
    const double s = 1.0 / sqrt(tot[0]);
    // the arguments live in LDS: a per-lane copy selected by the parity of
    // k would spill to scratch
    __shared__ PowerArgs a;
    if (flat_tid() == 0) {
        a = PowerArgs{};
        a.nx = I.nx;
        a.ny = I.ny;
        a.tiles_x = I.ptiles_x;
        a.tiles_y = I.ptiles_y;
        a.nb = I.nb;
        power_coeffs(I, a);
        a.in = (k == 0) ? (I.has_x0 ? I.x0 : I.y[1]) : I.y[(k - 1) & 1];
        a.out = I.y[k & 1];
        a.u = I.u;
    }
    __syncthreads();
    double acc = 0.0;
    const int T = I.ptiles_x * I.ptiles_y;
    // each thread marches down kBatchPowerRows rows, so a row of the input
    // is loaded once per tile instead of three times
    constexpr int RY = kBatchPowerRows;
    for_tile_band(T, I.nb, w.j, [&](int t) {
        if (I.kind == kOpDiffAdv) {
            if (I.vec == 2) power_tile<kOpDiffAdv, RY, 2>(a, s, acc, t);
            else power_tile<kOpDiffAdv, RY, 1>(a, s, acc, t);
        } else {
            if (I.vec == 2) power_tile<kOpBurgersJ, RY, 2>(a, s, acc, t);
            else power_tile<kOpBurgersJ, RY, 1>(a, s, acc, t);
        }
    });
    double v[1] = {acc};
    block_sum<1>(v);
    if (flat_tid() == 0) P[static_cast<long>(k & 1) * I.nb + w.j] = v[0];
}

// rho = ||w_P|| per instance, then lambda = -safety rho, c = lambda/2,
// gamma = -lambda/4 (Listing 7); one workgroup per instance
__global__ __launch_bounds__(kBlockThreads) void batch_power_final_kernel(BatchInst* insts,
                                                                          const double* partials,
                                                                          const int k_last, const double safety) {
    BatchInst& I = insts[blockIdx.x];
    double tot[1];
    sum_partials<1>(partials + I.part_off + static_cast<long>(k_last & 1) * I.nb, I.nb, tot);
    if (flat_tid() == 0) {
        const double rho = sqrt(tot[0]);
        const double lam = -safety * rho;
        I.rho = rho;
        I.c = lam / 2.0;
        I.gamma = -lam / 4.0;
        stencil_coeffs(I.kind == kOpDiffAdv ? 0 : 1, I.dx, I.dy, I.D, I.vx, I.vy, I.nu, I.c, I.gamma, I.st);
    }
}

// Newton coefficients d_0..d_{ld-1} of phi_l(h (c + gamma xi)) for one
// instance per workgroup of one wavefront: values at the Leja points in
// double-double, then the divided-difference table column by column
//     d_k <- (d_k - d_{k-1}) / (xi_k - xi_{k-j}),  k = ld-1 .. j,
// in chunks of 64 from the top, every chunk reading before it writes.
__global__ __launch_bounds__(kCoefThreads) void batch_coeffs_kernel(const BatchInst* insts,
                                                                    const double* __restrict__ xi,
                                                                    double* __restrict__ coef, const int ld) {
    __shared__ double hi[kMaxCoef], lo[kMaxCoef];
    const BatchInst& I = insts[blockIdx.x];
    const int lane = threadIdx.x;
    const int M = ld;
    for (int j = lane; j < M; j += kCoefThreads) {
        const dd f = dd_phi_at(I.l, 1.0, 1.0, I.h, I.c, I.gamma, xi[j]);
        hi[j] = f.hi;
        lo[j] = f.lo;
    }
    __syncthreads();
    for (int jj = 1; jj < M; ++jj) {
        for (int top = M - 1; top >= jj; top -= kCoefThreads) {
            const int k = top - lane;
            const bool act = k >= jj;
            dd nv{0.0, 0.0};
            if (act) {
                const dd a{hi[k], lo[k]}, b{hi[k - 1], lo[k - 1]};
                nv = dd_div(dd_sub(a, b), two_sum(xi[k], -xi[k - jj]));
            }
            __syncthreads();
            if (act) {
                hi[k] = nv.hi;
                lo[k] = nv.lo;
            }
            __syncthreads();
        }
    }
    for (int j = lane; j < M; j += kCoefThreads) coef[static_cast<long>(blockIdx.x) * ld + j] = hi[j] + lo[j];
}

__device__ __forceinline__ void sweep_coeffs(const BatchInst& I, SweepArgs& a) {
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
}

__global__ __launch_bounds__(kBlockThreads) void batch_sweep_kernel(const BatchInst* insts, LoopCtl* ctls,
                                                                    const int* block_inst, double* partials,
                                                                    const double* coef, const int ld,
                                                                    const double* xi, unsigned* done,
                                                                    const int m) {
    const Who w = who(insts, block_inst);
    const BatchInst& I = insts[w.i];
    LoopCtl* __restrict__ ctl = ctls + w.i;
    if (loop_ended(ctl)) return;
    // the instance's arguments live in LDS: a per-lane copy would be indexed
    // dynamically (the basis parity) and spill to scratch
    __shared__ SweepArgs a;
    const int tid = flat_tid();
    if (tid == 0) {
        a = SweepArgs{};
        a.nx = I.nx;
        a.ny = I.ny;
        a.tiles_x = I.tiles_x;
        a.tiles_y = I.tiles_y;
        a.nb = I.nb;
        a.ld = ld;
        sweep_coeffs(I, a);
        a.inv_sqrtN = 1.0 / sqrt(static_cast<double>(I.nx) * I.ny);
        a.v = I.v;
        a.ybuf[0] = I.y[0];
        a.ybuf[1] = I.y[1];
        a.u = I.u;
        a.u32 = nullptr;
        a.p[0] = I.out;
        a.coef = coef + static_cast<long>(w.i) * ld;
        a.xi = xi;
        a.partials = partials + I.part_off;
        a.ctl = ctl;
    }
    __syncthreads();

    __shared__ SweepState s_cur;
    if (m == 0) {
        if (tid == 0) s_cur = ctl->slot[0];
    } else {
        double tot[2];
        sum_partials<2>(gptr(a.partials) + static_cast<long>((m - 1) & 1) * I.nb * 2, I.nb, tot);
        if (tid == 0) {
            const SweepState nxt = decide<1, false>(a, *ctl, ctl->slot[(m - 1) & 1], m, tot);
            s_cur = nxt;
            if (w.j == 0) {
                ctl->slot[m & 1] = nxt;
                if (nxt.done) {
                    ctl->slot[2] = nxt;
                    atomicAdd(done, 1u);
                }
            }
        }
    }
    __syncthreads();
    if (s_cur.done) return;

    int act[1] = {s_cur.active[0]};
    double sy = 0.0, sp[1] = {0.0};
    const int T = I.tiles_x * I.tiles_y;
    for_tile_band(T, I.nb, w.j, [&](int t) {
        if (I.kind == kOpDiffAdv) {
            if (I.vec == 2) sweep_tile<kOpDiffAdv, 1, 1, 2, double, double, double>(a, m, act, sy, sp, t);
            else sweep_tile<kOpDiffAdv, 1, 1, 1, double, double, double>(a, m, act, sy, sp, t);
        } else {
            if (I.vec == 2) sweep_tile<kOpBurgersJ, 1, 1, 2, double, double, double>(a, m, act, sy, sp, t);
            else sweep_tile<kOpBurgersJ, 1, 1, 1, double, double, double>(a, m, act, sy, sp, t);
        }
    });

    double v[2] = {sy, sp[0]};
    block_sum<2>(v);
    if (tid == 0) {
        double* __restrict__ Pw = gptr(a.partials) + static_cast<long>(m & 1) * I.nb * 2 + w.j * 2;
        Pw[0] = v[0];
        Pw[1] = v[1];
    }
}

}  // namespace

hipError_t launch_batch_fill_x0(BatchInst* insts, const int* block_inst, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(batch_fill_x0_kernel, dim3(nblocks), dim3(kBatchTx, kBatchTy), 0, s, insts, block_inst);
    return hipGetLastError();
}

hipError_t launch_batch_power_norm(const BatchInst* insts, const int* block_inst, int nblocks, double* partials,
                                   hipStream_t s) {
    hipLaunchKernelGGL(batch_power_norm_kernel, dim3(nblocks), dim3(kBatchTx, kBatchTy), 0, s, insts, block_inst,
                       partials);
    return hipGetLastError();
}

hipError_t launch_batch_power_sweep(const BatchInst* insts, const int* block_inst, int nblocks, double* partials,
                                    int k, hipStream_t s) {
    hipLaunchKernelGGL(batch_power_sweep_kernel, dim3(nblocks), dim3(kBatchTx, kBatchTy), 0, s, insts, block_inst,
                       partials, k);
    return hipGetLastError();
}

hipError_t launch_batch_power_final(BatchInst* insts, int n_inst, const double* partials, int k_last,
                                    double safety, hipStream_t s) {
    hipLaunchKernelGGL(batch_power_final_kernel, dim3(n_inst), dim3(kBlockThreads), 0, s, insts, partials, k_last,
                       safety);
    return hipGetLastError();
}

hipError_t launch_batch_coeffs(const BatchInst* insts, int n_inst, const double* xi, double* coef, int ld,
                               hipStream_t s) {
    if (ld < 2 || ld > kMaxCoef) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_coeffs_kernel, dim3(n_inst), dim3(kCoefThreads), 0, s, insts, xi, coef, ld);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks,
                              double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                              int m, hipStream_t s) {
    hipLaunchKernelGGL(batch_sweep_kernel, dim3(nblocks), dim3(kBatchTx, kBatchTy), 0, s, insts, ctls, block_inst,
                       partials, coef, ld, xi, done, m);
    return hipGetLastError();
}

}  // namespace lx
