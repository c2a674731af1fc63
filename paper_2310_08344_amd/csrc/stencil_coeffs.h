// Coefficients of the periodic stencil operators, shared by the host
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

// Diffusion with third-order upwind advection (the gradient of Sec. 3):
// per axis with spacing d, speed v and Dd = D/d^2, the four-point
// upwind-biased first difference (exact for cubics) gives the upwind
// neighbour Dd + |v|/d, the downwind one Dd - |v|/(3d), the second upwind
// neighbour -|v|/(6d), the second downwind one 0 and the centre
// -2 Dd - |v|/(2d); "upwind" is the forward side for v >= 0.
//     out = {cE, cW, cN, cS, cC, cE2, cW2, cN2, cS2} of (A - c)/g.
LX_SHD void stencil_coeffs_up3(double dx, double dy, double D, double vx, double vy, double c, double g,
                               double (&out)[9]) {
    double ax[4], ay[4];   // {E, W, E2, W2} along x, {N, S, N2, S2} along y
    const double sp[2] = {vx, vy}, dd[2] = {dx, dy};
    for (int t = 0; t < 2; ++t) {
        double* o = t == 0 ? ax : ay;
        const double d = dd[t], a = sp[t] < 0.0 ? -sp[t] : sp[t], Dd = D / (d * d);
        const double up = Dd + a / d, down = Dd - a / (3.0 * d), up2 = -a / (6.0 * d);
        if (sp[t] >= 0.0) {
            o[0] = up;
            o[1] = down;
            o[2] = up2;
            o[3] = 0.0;
        } else {
            o[0] = down;
            o[1] = up;
            o[2] = 0.0;
            o[3] = up2;
        }
    }
    const double cC = -(2.0 * D / (dx * dx) + 2.0 * D / (dy * dy)) -
                      ((vx < 0.0 ? -vx : vx) / (2.0 * dx) + (vy < 0.0 ? -vy : vy) / (2.0 * dy));
    out[0] = ax[0] / g;
    out[1] = ax[1] / g;
    out[2] = ay[0] / g;
    out[3] = ay[1] / g;
    out[4] = (cC - c) / g;
    out[5] = ax[2] / g;
    out[6] = ax[3] / g;
    out[7] = ay[2] / g;
    out[8] = ay[3] / g;
}

}  // namespace lx
