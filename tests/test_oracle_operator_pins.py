"""Pins of the oracle's stencils against facts fixed outside the oracle.

* Diffusion-advection: every 2-D Fourier mode is an eigenvector whose
  eigenvalue is the analytic symbol of the centred Laplacian plus the
  first-order upwind difference (each side of the upwind switch is hit);
  every symbol has a non-positive real part (Sec. 2.1 needs the spectrum in
  the left half plane); the periodic stencil conserves the sum.
* Burgers: F is quadratic, so (F(u + e w) - F(u - e w)) / (2 e) equals J(u) w
  up to rounding; both conserve the sum; with u constant, J(u) acts on a
  Fourier mode by its analytic symbol.
* The closed-form spectral radius of the diffusion-advection stencil equals
  the largest eigenvalue modulus of the assembled matrix.
"""
import numpy as np
import pytest

from oracle.exact import dense_matrix, diffadv_symbol
from oracle.operators import burgers_F, burgers_J, diffadv_apply
from paper_2310_08344_amd.workloads import diffadv_cfl_step


def _mode(ny, nx, kx, ky):
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.exp(2j * np.pi * (kx * i / nx + ky * j / ny))


@pytest.mark.parametrize("vx,vy", [(3.0, 5.0), (-4.0, 2.0), (1.5, -0.5), (-2.0, -7.0), (0.0, 0.0)])
def test_diffadv_fourier_modes_are_eigenvectors(vx, vy):
    ny, nx = 6, 10
    D, dx, dy = 0.7, 1.0 / 10, 1.0 / 6
    lam = diffadv_symbol(ny, nx, D, vx, vy, dx, dy)
    for kx in range(nx):
        for ky in range(ny):
            m = _mode(ny, nx, kx, ky)
            got = diffadv_apply(m, D, vx, vy, dx, dy)
            # hand-written symbol of this mode (independent of diffadv_symbol)
            tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
            ref = D * (2 * np.cos(tx) - 2) / dx**2 + D * (2 * np.cos(ty) - 2) / dy**2
            ref += vx * ((np.exp(1j * tx) - 1) if vx >= 0 else (1 - np.exp(-1j * tx))) / dx
            ref += vy * ((np.exp(1j * ty) - 1) if vy >= 0 else (1 - np.exp(-1j * ty))) / dy
            assert np.allclose(got, ref * m, rtol=0, atol=1e-10 * max(1.0, abs(ref)))
            kxs = kx if kx <= nx // 2 else kx - nx   # fftfreq layout
            kys = ky if ky <= ny // 2 else ky - ny
            assert abs(lam[kys % ny, kxs % nx] - ref) <= 1e-10 * max(1.0, abs(ref))
            assert ref.real <= 1e-12


def test_diffadv_conserves_sum():
    rng = np.random.default_rng(0)
    y = rng.standard_normal((12, 16))
    out = diffadv_apply(y, 1.3, 2.0, -3.0, 1 / 16, 1 / 12)
    assert abs(out.sum()) <= 1e-11 * np.abs(out).sum()


@pytest.mark.parametrize("D,vx,vy,n", [(1.0, 8.0, 8.0, 8), (0.3, -2.0, 5.0, 8), (2.0, 0.5, 0.0, 6)])
def test_closed_form_spectral_radius(D, vx, vy, n):
    A = dense_matrix(lambda y: diffadv_apply(y, D, vx, vy, 1 / n, 1 / n), n, n)
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    rho_closed = 2.0 / diffadv_cfl_step(D, vx, vy, 1 / n, 1 / n)
    # Gershgorin bound, attained by the real eigenvalue of the (pi, pi) mode
    # (n even)
    assert abs(rho - rho_closed) <= 1e-10 * rho_closed


def test_burgers_jacobian_is_exact_derivative_of_F():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((9, 14))
    w = rng.standard_normal((9, 14))
    nu, dx, dy = 0.02, 1 / 14, 1 / 9
    for e in (1e-2, 1e-4):
        fd = (burgers_F(u + e * w, nu, dx, dy) - burgers_F(u - e * w, nu, dx, dy)) / (2 * e)
        jw = burgers_J(u, w, nu, dx, dy)
        assert np.max(np.abs(fd - jw)) <= 1e-8 * np.max(np.abs(jw))


def test_burgers_conserves_sum_and_kills_constants():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((8, 8))
    w = rng.standard_normal((8, 8))
    nu, dx = 0.01, 1 / 8
    assert abs(burgers_F(u, nu, dx, dx).sum()) <= 1e-12 * np.abs(burgers_F(u, nu, dx, dx)).sum()
    assert abs(burgers_J(u, w, nu, dx, dx).sum()) <= 1e-12 * np.abs(burgers_J(u, w, nu, dx, dx)).sum()
    assert np.max(np.abs(burgers_F(np.full((8, 8), 3.0), nu, dx, dx))) <= 1e-12


def test_burgers_jacobian_symbol_at_constant_state():
    ny, nx = 8, 12
    U, nu, dx, dy = 1.7, 0.05, 1 / 12, 1 / 8
    u = np.full((ny, nx), U)
    for kx, ky in [(1, 0), (3, 2), (5, 7), (6, 4)]:
        m = _mode(ny, nx, kx, ky)
        tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
        ref = nu * ((2 * np.cos(tx) - 2) / dx**2 + (2 * np.cos(ty) - 2) / dy**2)
        ref -= U * (1j * np.sin(tx) / dx + 1j * np.sin(ty) / dy)
        got = burgers_J(u, m, nu, dx, dy)
        assert np.allclose(got, ref * m, rtol=0, atol=1e-10 * abs(ref))
