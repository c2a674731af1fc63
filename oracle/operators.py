"""Periodic 2-D stencil operators (oracle side), written with numpy.roll.

TEST INFRASTRUCTURE ONLY (see the package header).

Arrays are [ny, nx]: axis 1 is x (index i), axis 0 is y (index j).

Diffusion-advection (Sec. 3, Eq. (3) with the paper's sign of the advection
term, u_t = D lap(u) + v . grad(u)):
  * the Laplacian is the second-order centred 5-point stencil (Sec. 3);
  * grad is first-order upwind (reading: the benchmark workloads name a
    first-order upwind gradient; the paper's own third-order scheme is the
    next operator below).  The side is chosen so that every eigenvalue has a
    non-positive real part, which the Leja interval of Sec. 2.1 assumes:
    v > 0 takes the forward difference (u_{i+1} - u_i)/dx, v < 0 the
    backward one.

Diffusion-advection with the paper's own gradient (Sec. 3: the gradient is
discretised by a third-order upwind scheme, the Laplacian by the centred
second-order one): the first derivative is the four-point upwind-biased
difference that is exact for cubics.  For v >= 0 the stencil leans to the
forward side (points i-1 .. i+2),
    d_x y ~ (-y_{i+2} + 6 y_{i+1} - 3 y_i - 2 y_{i-1}) / (6 dx),
and for v < 0 it is mirrored (points i-2 .. i+1),
    d_x y ~ (2 y_{i+1} + 3 y_i - 6 y_{i-1} + y_{i-2}) / (6 dx),
the side on which every Fourier mode decays (the real part of v times the
difference's symbol is -|v| (1 - cos t)^2 / (3 dx) <= 0).

Burgers (Sec. 3, Eq. (5), in the viscous conservative form used by the
benchmark workloads): F(u) = nu lap(u) - (1/2)[d_x(u^2) + d_y(u^2)] with
centred first differences; its Jacobian is
J(u) w = nu lap(w) - [d_x(u w) + d_y(u w)].
"""
from __future__ import annotations

import numpy as np


def _east(y):
    return np.roll(y, -1, axis=1)   # y[j, i+1]


def _west(y):
    return np.roll(y, 1, axis=1)    # y[j, i-1]


def _north(y):
    return np.roll(y, -1, axis=0)   # y[j+1, i]


def _south(y):
    return np.roll(y, 1, axis=0)    # y[j-1, i]


def laplacian(y, dx, dy):
    return (_east(y) - 2.0 * y + _west(y)) / dx**2 + (_north(y) - 2.0 * y + _south(y)) / dy**2


def upwind(y, vx, vy, dx, dy):
    if vx >= 0.0:
        ax = vx * (_east(y) - y) / dx
    else:
        ax = vx * (y - _west(y)) / dx
    if vy >= 0.0:
        ay = vy * (_north(y) - y) / dy
    else:
        ay = vy * (y - _south(y)) / dy
    return ax + ay


def _d3(y, axis, v, d):
    """v times the third-order upwind-biased first difference along axis."""
    p1 = np.roll(y, -1, axis=axis)
    p2 = np.roll(y, -2, axis=axis)
    m1 = np.roll(y, 1, axis=axis)
    m2 = np.roll(y, 2, axis=axis)
    if v >= 0.0:
        return v * (-p2 + 6.0 * p1 - 3.0 * y - 2.0 * m1) / (6.0 * d)
    return v * (2.0 * p1 + 3.0 * y - 6.0 * m1 + m2) / (6.0 * d)


def upwind3(y, vx, vy, dx, dy):
    return _d3(y, 1, vx, dx) + _d3(y, 0, vy, dy)


def diffadv3_apply(y, D, vx, vy, dx, dy):
    """A y for A = D*Laplacian + v . (third-order upwind gradient), periodic."""
    return D * laplacian(y, dx, dy) + upwind3(y, vx, vy, dx, dy)


def diffadv_apply(y, D, vx, vy, dx, dy):
    """A y for A = D*Laplacian + v . (upwind gradient), periodic."""
    return D * laplacian(y, dx, dy) + upwind(y, vx, vy, dx, dy)


def centred_div(f, dx, dy):
    """d_x f + d_y f with centred first differences."""
    return (_east(f) - _west(f)) / (2.0 * dx) + (_north(f) - _south(f)) / (2.0 * dy)


def burgers_F(u, nu, dx, dy):
    """F(u) = nu lap(u) - (1/2)(d_x + d_y)(u^2)."""
    return nu * laplacian(u, dx, dy) - 0.5 * centred_div(u * u, dx, dy)


def burgers_J(u, w, nu, dx, dy):
    """Analytic Jacobian action J(u) w = nu lap(w) - (d_x + d_y)(u w)."""
    return nu * laplacian(w, dx, dy) - centred_div(u * w, dx, dy)


def make_apply(problem, u=None):
    """Linear map y -> A y for a workload Problem (Jacobian at u for Burgers)."""
    dx, dy = problem.dx, problem.dy
    if problem.kind == "diffadv":
        return lambda y: diffadv_apply(y, problem.D, problem.vx, problem.vy, dx, dy)
    if problem.kind == "diffadv3":
        return lambda y: diffadv3_apply(y, problem.D, problem.vx, problem.vy, dx, dy)
    if problem.kind == "burgers":
        if u is None:
            raise ValueError("Burgers Jacobian needs the state u")
        return lambda w: burgers_J(u, w, problem.nu, dx, dy)
    raise ValueError(problem.kind)
