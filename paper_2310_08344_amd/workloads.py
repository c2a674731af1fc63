"""Seeded synthetic workloads for the Leja phi-action path.

This module only draws inputs: grids, operator parameters, initial data and
step sizes.  It holds none of the method's arithmetic (no Leja points, no
phi functions, no divided differences, no stencil application), so both the
HIP path and the CPU oracle can take their inputs from it.

Conventions shared by every workload:

* the domain is the periodic unit square [0, 1)^2 with ``n x n`` cells,
  ``dx = dy = 1/n`` and grid points ``x_i = i*dx`` (the paper-shaped linear
  problems use [-1, 1)^2: ``dx = 2/n``, ``x_i = -1 + i*dx``);
* arrays are row-major ``[ny][nx]``: the x index is the fast one;
* the step size is a multiple ``s`` of the explicit CFL step, read as
  ``2 / rho`` where ``rho`` bounds the modulus of the discrete operator's
  spectrum (Gershgorin; the paper uses Delta t_CFL in Sec. 3 without defining
  it).  For the diffusion-advection stencil this bound is attained.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

DIFFADV = "diffadv"
DIFFADV3 = "diffadv3"   # diffusion + third-order upwind advection
BURGERS = "burgers"


@dataclass
class Problem:
    """One phi-action problem instance (operator parameters + data)."""

    kind: str
    n: int
    D: float = 0.0          # diffusion coefficient (diffusion-advection)
    vx: float = 0.0         # advection velocity, x
    vy: float = 0.0         # advection velocity, y
    nu: float = 0.0         # viscosity (Burgers)
    h: float = 0.0          # time step
    cfl_multiple: float = 0.0
    seed: int = 0
    meta: dict = field(default_factory=dict)
    length: float = 1.0     # side of the periodic square

    @property
    def dx(self) -> float:
        return self.length / self.n

    @property
    def dy(self) -> float:
        return self.length / self.n

    @property
    def N(self) -> int:
        return self.n * self.n

    def params(self) -> dict:
        d = asdict(self)
        d["dx"] = self.dx
        d["dy"] = self.dy
        return d


# --------------------------------------------------------------------------
# step-size rule (problem definition, not part of the method)
# --------------------------------------------------------------------------

def diffadv_cfl_step(D: float, vx: float, vy: float, dx: float, dy: float) -> float:
    """Explicit CFL step 2/rho of the periodic diffusion + first-order upwind
    stencil, rho = 4D/dx^2 + 4D/dy^2 + 2|vx|/dx + 2|vy|/dy."""
    rho = 4.0 * D / dx**2 + 4.0 * D / dy**2 + 2.0 * abs(vx) / dx + 2.0 * abs(vy) / dy
    return 2.0 / rho


def diffadv3_cfl_step(D: float, vx: float, vy: float, dx: float, dy: float) -> float:
    """Explicit CFL step 2/rho with rho the Gershgorin bound (row sum of
    moduli) of the periodic diffusion + third-order upwind stencil: per axis
    with spacing d and speed |v|, the centre 2D/d^2 + |v|/(2d) and the
    neighbours |D/d^2 - |v|/(3d)|, D/d^2 + |v|/d and |v|/(6d)."""
    rho = 0.0
    for v, d in ((abs(vx), dx), (abs(vy), dy)):
        rho += 2.0 * D / d**2 + v / (2.0 * d) + abs(D / d**2 - v / (3.0 * d)) + D / d**2 + v / d + v / (6.0 * d)
    return 2.0 / rho


def burgers_cfl_step(nu: float, umax: float, dx: float, dy: float) -> float:
    """Explicit CFL step 2/rho_b for the Burgers Jacobian with centred
    differences, rho_b = 4 nu/dx^2 + 4 nu/dy^2 + |u|_max (1/dx + 1/dy)."""
    rho = 4.0 * nu / dx**2 + 4.0 * nu / dy**2 + umax * (1.0 / dx + 1.0 / dy)
    return 2.0 / rho


# --------------------------------------------------------------------------
# initial data
# --------------------------------------------------------------------------

def grid(n: int):
    x = np.arange(n, dtype=np.float64) / n
    return np.meshgrid(x, x, indexing="xy")  # X[j, i] = x_i, Y[j, i] = y_j


def gaussian(n: int, cx: float = 0.5, cy: float = 0.5, sigma: float = 0.1) -> np.ndarray:
    """exp(-((x-cx)^2 + (y-cy)^2)/sigma^2) on the grid (no periodic images)."""
    X, Y = grid(n)
    return np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / sigma**2)


def random_normal(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n, n))


def fourier_modes(n: int, seed: int, n_modes: int = 4, kmax: int = 4) -> np.ndarray:
    """sum_k a_k sin(2 pi (m_k x + n_k y) + theta_k), a_k ~ U(0,1),
    (m_k, n_k) uniform integers in [-kmax, kmax]^2 minus the origin,
    theta_k ~ U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    X, Y = grid(n)
    u = np.zeros((n, n))
    for _ in range(n_modes):
        a = rng.uniform(0.0, 1.0)
        while True:
            m, k = rng.integers(-kmax, kmax + 1, size=2)
            if m != 0 or k != 0:
                break
        th = rng.uniform(0.0, 2.0 * math.pi)
        u += a * np.sin(2.0 * math.pi * (m * X + k * Y) + th)
    return u


def start_vector(n: int, seed: int = 12345) -> np.ndarray:
    """Seeded N(0,1) start vector for power iteration (a constant vector is
    invalid: it lies in the null space of the periodic operators)."""
    return np.random.default_rng(seed).standard_normal((n, n))


# --------------------------------------------------------------------------
# the five workload families
# --------------------------------------------------------------------------

def config1(n: int = 64) -> tuple[Problem, np.ndarray]:
    """Periodic 64^2 diffusion-advection, D = 1, cell Peclet number 1 per
    component (v = (D/dx)(1, 1)), centred Gaussian (sigma = 0.1),
    h = 10 x CFL; exp(hA)u at rtol 1e-10."""
    dx = 1.0 / n
    D = 1.0
    v = D / dx
    h = 10.0 * diffadv_cfl_step(D, v, v, dx, dx)
    p = Problem(DIFFADV, n, D=D, vx=v, vy=v, h=h, cfl_multiple=10.0,
                meta={"l": [0], "rtol": 1e-10, "atol": 0.0, "power_iters": 20})
    return p, gaussian(n)


def config2(n: int = 1024, seed: int | None = None) -> tuple[Problem, np.ndarray]:
    """Same operator family at paper scale, h = 50 x CFL, phi_1..phi_3 of a
    seeded N(0,1) vector at rtol 1e-8 (seed 1 for 1024^2, 2 for 4096^2)."""
    if seed is None:
        seed = {1024: 1, 4096: 2}.get(n, 7)
    dx = 1.0 / n
    D = 1.0
    v = D / dx
    h = 50.0 * diffadv_cfl_step(D, v, v, dx, dx)
    p = Problem(DIFFADV, n, D=D, vx=v, vy=v, h=h, cfl_multiple=50.0, seed=seed,
                meta={"l": [1, 2, 3], "rtol": 1e-8, "atol": 0.0, "power_iters": 20})
    return p, random_normal(n, seed)


def config3(n: int = 2048, seed: int = 3, nu: float = 1e-3,
            cfl_multiple: float = 10.0) -> tuple[Problem, np.ndarray]:
    """Periodic viscous Burgers, u0 = 4 seeded Fourier modes, one EXPRB42
    step of size h = 10 x CFL of the Jacobian at u0, rtol 1e-8."""
    u0 = fourier_modes(n, seed)
    dx = 1.0 / n
    h = cfl_multiple * burgers_cfl_step(nu, float(np.max(np.abs(u0))), dx, dx)
    p = Problem(BURGERS, n, nu=nu, h=h, cfl_multiple=cfl_multiple, seed=seed,
                meta={"rtol": 1e-8, "atol": 0.0, "power_iters": 20})
    return p, u0


def batched_instances(count: int = 256, seed: int = 4,
                      sizes=(64, 128, 256, 512), s_range=(1.0, 50.0)) -> list[tuple[Problem, np.ndarray]]:
    """Independent diffusion-advection instances with uneven work: grid side
    uniform over ``sizes``, D ~ LogU(0.1, 10), |v| ~ U(0, 5) with a random
    direction, Gaussian (sigma 0.1) at a random centre, h = s x CFL with
    s ~ LogU(s_range); exp action at rtol 1e-8."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        D = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        speed = float(rng.uniform(0.0, 5.0))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        s = float(math.exp(rng.uniform(math.log(s_range[0]), math.log(s_range[1]))))
        dx = 1.0 / n
        vx, vy = speed * math.cos(ang), speed * math.sin(ang)
        h = s * diffadv_cfl_step(D, vx, vy, dx, dx)
        p = Problem(DIFFADV, n, D=D, vx=vx, vy=vy, h=h, cfl_multiple=s, seed=seed,
                    meta={"index": i, "l": [0], "rtol": 1e-8, "atol": 0.0,
                          "speed": speed, "angle": ang})
        out.append((p, gaussian(n, float(cx), float(cy))))
    return out


def paper_linear(n: int = 8192, cfl_multiple: float = 1.0, source: bool = False,
                 rtol: float = 1e-12) -> tuple[Problem, np.ndarray, np.ndarray | None]:
    """The paper's linear test problems (Sec. 3, Problems I and II) on the
    periodic square [-1, 1)^2 with n x n cells: u_t = lap(u) + nu (u_x + u_y)
    with nu = 10, the Laplacian centred and the gradient third-order upwind;
    u0 = 1 + exp(-((x + 0.5)^2 + (y + 0.5)^2)/0.01).  With ``source`` the
    time-independent source S = exp(-((x + 0.4)^2 + (y - 0.6)^2)/0.05)
    + exp(-((x - 0.25)^2 + (y + 0.1)^2)/0.04) is added (Problem II).
    h = cfl_multiple x CFL; tolerance 1e-12 as in every run of the paper.
    Returns (problem, u0, S or None)."""
    L = 2.0
    dx = L / n
    nu = 10.0
    x = -1.0 + np.arange(n, dtype=np.float64) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = 1.0 + np.exp(-((X + 0.5) ** 2 + (Y + 0.5) ** 2) / 0.01)
    S = None
    if source:
        S = np.exp(-((X + 0.4) ** 2 + (Y - 0.6) ** 2) / 0.05) + np.exp(-((X - 0.25) ** 2 + (Y + 0.1) ** 2) / 0.04)
    h = cfl_multiple * diffadv3_cfl_step(1.0, nu, nu, dx, dx)
    p = Problem(DIFFADV3, n, D=1.0, vx=nu, vy=nu, h=h, cfl_multiple=cfl_multiple, length=L,
                meta={"rtol": rtol, "atol": 0.0, "power_iters": 20, "problem": "II" if source else "I"})
    return p, u0, S


def learned_instance(index: int, seed0: int, sizes=(64, 128, 256)):
    """One instance of the predictor's training/evaluation distribution,
    drawn from its own seed (seed0 + index).  Even indices: diffusion-
    advection as in ``batched_instances`` (Gaussian input), h = s x CFL with
    s ~ LogU(1, 100); odd indices: Burgers with a four-mode Fourier state u,
    whose Jacobian acts on v = u, viscosity from the cell Peclet number
    Pe = max|u| dx / nu ~ LogU(1/4, 4) and h = s x CFL with s ~ LogU(1, 10);
    phi order l ~ U{0..3}.  (Reading: interpolation at real Leja points needs
    the Jacobian's spectrum close to the negative real axis; at cell Peclet
    numbers well above 2 the centred Burgers Jacobian is advection-dominated,
    its spectrum nearly imaginary, and the plain method diverges, so the
    distribution keeps to the diffusion-dominated regime of the Burgers
    workload at 2048^2, where Pe is about 2.)
    Returns (Problem, u or None, v)."""
    rng = np.random.default_rng(seed0 + index)
    n = int(rng.choice(sizes))
    dx = 1.0 / n
    l = int(rng.integers(0, 4))
    if index % 2 == 0:
        D = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        speed = float(rng.uniform(0.0, 5.0))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        s = float(math.exp(rng.uniform(0.0, math.log(100.0))))
        vx, vy = speed * math.cos(ang), speed * math.sin(ang)
        h = s * diffadv_cfl_step(D, vx, vy, dx, dx)
        p = Problem(DIFFADV, n, D=D, vx=vx, vy=vy, h=h, cfl_multiple=s, seed=seed0 + index,
                    meta={"l": l, "index": index})
        return p, None, gaussian(n, float(cx), float(cy))
    pe = float(math.exp(rng.uniform(math.log(0.25), math.log(4.0))))
    s = float(math.exp(rng.uniform(0.0, math.log(10.0))))
    u = fourier_modes(n, int(rng.integers(0, 2**31 - 1)))
    umax = float(np.max(np.abs(u)))
    nu = umax * dx / pe
    h = s * burgers_cfl_step(nu, umax, dx, dx)
    p = Problem(BURGERS, n, nu=nu, h=h, cfl_multiple=s, seed=seed0 + index, meta={"l": l, "index": index})
    return p, u, u.copy()
