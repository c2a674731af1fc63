// Coefficients of the two periodic five-point operators, shared by the host
// and by device code that derives them from a shift computed on the device.
//
// Diffusion-advection (second-order diffusion, first-order upwind
// advection chosen so that the spectrum has a non-positive real part):
//     (A y)_C = cE y_E + cW y_W + cN y_N + cS y_S + cC y_C,
// Burgers Jacobian at u (centred differences of nu Lap w - div(u w) / 1,
// with the flux of (1/2) u^2):
//     (J w)_C = kx (w_E + w_W) + ky (w_N + w_S) - gx (u_E w_E - u_W w_W)
//               - gy (u_N w_N - u_S w_S) + kC w_C,   kC = -2 kx - 2 ky.
#pragma once

#if defined(__HIPCC__)
#define LX_SHD __host__ __device__ inline
#else
#define LX_SHD inline
#endif

namespace lx {

// out = {cE, cW, cN, cS, cC} (kind 0) or {kx, ky, gx, gy, kC} (kind 1) of
// the operator (A - c)/g; the plain operator is c = 0, g = 1.
LX_SHD void stencil_coeffs(int kind, double dx, double dy, double D, double vx, double vy, double nu, double c,
                           double g, double (&out)[5]) {
    if (kind == 0) {
        const double ex = D / (dx * dx), ey = D / (dy * dy);
        const double cE = ex + (vx > 0.0 ? vx : 0.0) / dx, cW = ex + (vx < 0.0 ? -vx : 0.0) / dx;
        const double cN = ey + (vy > 0.0 ? vy : 0.0) / dy, cS = ey + (vy < 0.0 ? -vy : 0.0) / dy;
        const double cC = -(cE + cW + cN + cS);
        out[0] = cE / g;
        out[1] = cW / g;
        out[2] = cN / g;
        out[3] = cS / g;
        out[4] = (cC - c) / g;
    } else {
        out[0] = nu / (g * dx * dx);
        out[1] = nu / (g * dy * dy);
        out[2] = 1.0 / (2.0 * g * dx);
        out[3] = 1.0 / (2.0 * g * dy);
        out[4] = -2.0 * out[0] - 2.0 * out[1] - c / g;
    }
}

}  // namespace lx
