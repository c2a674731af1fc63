// Tile building blocks of the multi-iteration Leja kernels (pair.hip,
// block.hip): 128-column tiles staged in LDS, the stencils of the shifted
// operator on LDS rows, and the launch arguments a tile reads.
#pragma once

#include <hip/hip_runtime.h>

#include "lx_device.h"
#include "sweep_device.h"

namespace lx {
namespace dev {

constexpr int kPairTW = 128;                // tile columns
constexpr int kPairWaves = kBlockThreads / 64;

template <int OP>
constexpr int radius() {
    return OP == kOpDiffAdv3 ? 2 : 1;
}
// LDS row pitch in doubles: the tile and a 2R halo on each side (a 16-byte
// multiple)
template <int R>
constexpr int pitch() {
    return kPairTW + 4 * R;
}

// the outputs are read and written once per launch: streaming
// (nontemporal) accesses that leave the caches to the basis vector
__device__ __forceinline__ double2 ld_stream(const double* p) {
    double v[2];
    ldv_nt<2>(p, v);
    double2 r;
    r.x = v[0];
    r.y = v[1];
    return r;
}
__device__ __forceinline__ void st_stream(double* p, const double2 t) {
    const double v[2] = {t.x, t.y};
    stv_nt<2>(p, v);
}

// The stencil of (A - c)/gamma: aW, aE, aS, aN, aC (diffusion-advection;
// third-order upwind adds aW2, aE2, aS2, aN2 in e0..e3) or kx, ky, gx, gy, kC
// (Burgers).
struct Sten {
    double c0, c1, c2, c3, c4;
    double e0, e1, e2, e3;
};

// What the tile code reads of the launch arguments, held in registers for
// the whole launch (the batched kernel keeps its SweepArgs in LDS, where a
// read after any LDS store would be issued again).
template <int K>
struct TileArgs {
    int nx, ny, tiles_x, ld;
    Sten st;
    const double* u;
    const double* coef;
    const double* xi;
    double* p[K];
};

template <int OP, int K>
__device__ __forceinline__ TileArgs<K> tile_args(const SweepArgs& a) {
    TileArgs<K> t;
    t.nx = a.nx;
    t.ny = a.ny;
    t.tiles_x = a.tiles_x;
    t.ld = a.ld;
    if constexpr (OP == kOpDiffAdv) {
        t.st = Sten{a.aW, a.aE, a.aS, a.aN, a.aC, 0.0, 0.0, 0.0, 0.0};
    } else if constexpr (OP == kOpDiffAdv3) {
        t.st = Sten{a.aW, a.aE, a.aS, a.aN, a.aC, a.aW2, a.aE2, a.aS2, a.aN2};
    } else {
        t.st = Sten{a.kx, a.ky, a.gx, a.gy, a.kC, 0.0, 0.0, 0.0, 0.0};
    }
    t.u = gptr(a.u);
    t.coef = gptr(a.coef);
    t.xi = gptr(a.xi);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        t.p[k] = gptr(a.p[k]);
    }
    return t;
}

// The shifted operator at one point from its four neighbours (W, E, S, N),
// its centre C and, for Burgers, u at the same cells: the stencils of the
// single-sweep kernel, so both compute the same bits.
template <int OP>
__device__ __forceinline__ double shifted_at(const Sten& k, const double shift, double W, double E, double S,
                                             double N, double C, double uW, double uE, double uS, double uN) {
    if constexpr (OP == kOpDiffAdv) {
        return stencil_da(k.c0, k.c1, k.c2, k.c3, k.c4 - shift, W, E, S, N, C);
    } else {
        return stencil_bu(k.c0, k.c1, k.c2, k.c3, k.c4 - shift, W, E, S, N, C, uW, uE, uS, uN);
    }
}

// the operator on LDS row `ce` (rows `up`, `dn` above and below) at the
// column pair j, j+1 (j even)
template <int OP>
__device__ __forceinline__ void shifted_pair(const Sten& a, const double shift, const double* up,
                                             const double* ce, const double* dn, const double* uup,
                                             const double* uce, const double* udn, const int j, double (&o)[2]) {
    const double2 c2 = *reinterpret_cast<const double2*>(ce + j);
    const double2 u2 = *reinterpret_cast<const double2*>(up + j);
    const double2 d2 = *reinterpret_cast<const double2*>(dn + j);
    const double l = ce[j - 1], r = ce[j + 2];
    if constexpr (OP == kOpDiffAdv) {
        o[0] = shifted_at<OP>(a, shift, l, c2.y, u2.x, d2.x, c2.x, 0, 0, 0, 0);
        o[1] = shifted_at<OP>(a, shift, c2.x, r, u2.y, d2.y, c2.y, 0, 0, 0, 0);
    } else {
        const double2 uc = *reinterpret_cast<const double2*>(uce + j);
        const double2 uu = *reinterpret_cast<const double2*>(uup + j);
        const double2 ud = *reinterpret_cast<const double2*>(udn + j);
        const double ul = uce[j - 1], ur = uce[j + 2];
        o[0] = shifted_at<OP>(a, shift, l, c2.y, u2.x, d2.x, c2.x, ul, uc.y, uu.x, ud.x);
        o[1] = shifted_at<OP>(a, shift, c2.x, r, u2.y, d2.y, c2.y, uc.x, ur, uu.y, ud.y);
    }
}

template <int OP>
__device__ __forceinline__ double shifted_one(const Sten& a, const double shift, const double* up,
                                              const double* ce, const double* dn, const double* uup,
                                              const double* uce, const double* udn, const int j) {
    if constexpr (OP == kOpDiffAdv) {
        return shifted_at<OP>(a, shift, ce[j - 1], ce[j + 1], up[j], dn[j], ce[j], 0, 0, 0, 0);
    } else {
        return shifted_at<OP>(a, shift, ce[j - 1], ce[j + 1], up[j], dn[j], ce[j], uce[j - 1], uce[j + 1], uup[j],
                              udn[j]);
    }
}

// the radius-2 operator on LDS row ce (rows u2, u1 below and d1, d2 above)
// at the column pair j, j+1 (j even), and at the single column j
__device__ __forceinline__ void shifted_pair3(const Sten& a, const double shift, const double* u2, const double* u1,
                                              const double* ce, const double* d1, const double* d2, const int j,
                                              double (&o)[2]) {
    const double2 c2 = *reinterpret_cast<const double2*>(ce + j);
    const double2 s1 = *reinterpret_cast<const double2*>(u1 + j);
    const double2 s2 = *reinterpret_cast<const double2*>(u2 + j);
    const double2 n1 = *reinterpret_cast<const double2*>(d1 + j);
    const double2 n2 = *reinterpret_cast<const double2*>(d2 + j);
    const double l1 = ce[j - 1], l2 = ce[j - 2], r1 = ce[j + 2], r2 = ce[j + 3];
    const double cc = a.c4 - shift;
    o[0] = stencil_d3(a.c0, a.c1, a.c2, a.c3, cc, a.e0, a.e1, a.e2, a.e3, l1, c2.y, s1.x, n1.x, c2.x, l2, r1, s2.x,
                      n2.x);
    o[1] = stencil_d3(a.c0, a.c1, a.c2, a.c3, cc, a.e0, a.e1, a.e2, a.e3, c2.x, r1, s1.y, n1.y, c2.y, l1, r2, s2.y,
                      n2.y);
}

__device__ __forceinline__ double shifted_one3(const Sten& a, const double shift, const double* u2, const double* u1,
                                               const double* ce, const double* d1, const double* d2, const int j) {
    return stencil_d3(a.c0, a.c1, a.c2, a.c3, a.c4 - shift, a.e0, a.e1, a.e2, a.e3, ce[j - 1], ce[j + 1], u1[j], d1[j],
                      ce[j], ce[j - 2], ce[j + 2], u2[j], d2[j]);
}

}  // namespace dev
}  // namespace lx
