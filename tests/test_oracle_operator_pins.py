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
* Diffusion + third-order upwind advection: Fourier modes are eigenvectors
  with a symbol written in real/imaginary form by hand; the difference is
  exact for cubics away from the seam and third order on a smooth periodic
  function; the CFL rule is the assembled matrix's Gershgorin bound and
  covers its spectrum; the sum is conserved.
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


# ---- diffusion + third-order upwind advection (Sec. 3) -------------------

@pytest.mark.parametrize("vx,vy", [(3.0, 5.0), (-4.0, 2.0), (1.5, -0.5), (-2.0, -7.0), (0.0, 0.0)])
def test_diffadv3_fourier_modes_are_eigenvectors(vx, vy):
    from oracle.exact import diffadv3_symbol
    from oracle.operators import diffadv3_apply
    ny, nx = 7, 10
    D, dx, dy = 0.7, 1.0 / 10, 1.0 / 7
    lam = diffadv3_symbol(ny, nx, D, vx, vy, dx, dy)
    for kx in range(nx):
        for ky in range(ny):
            m = _mode(ny, nx, kx, ky)
            got = diffadv3_apply(m, D, vx, vy, dx, dy)
            # hand-written symbol in real/imaginary form: the four-point
            # upwind difference has imaginary part (8 sin t - sin 2t)/6 and
            # damping -(1 - cos t)^2/3 on the upwind side
            tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
            ref = D * (2 * np.cos(tx) - 2) / dx**2 + D * (2 * np.cos(ty) - 2) / dy**2
            for v, t, d in ((vx, tx, dx), (vy, ty, dy)):
                ref += (1j * v * (8 * np.sin(t) - np.sin(2 * t)) / 6 - abs(v) * (1 - np.cos(t)) ** 2 / 3) / d
            assert np.allclose(got, ref * m, rtol=0, atol=1e-10 * max(1.0, abs(ref)))
            kxs = kx if kx <= nx // 2 else kx - nx
            kys = ky if ky <= ny // 2 else ky - ny
            assert abs(lam[kys % ny, kxs % nx] - ref) <= 1e-10 * max(1.0, abs(ref))
            assert ref.real <= 1e-12


@pytest.mark.parametrize("v", [2.5, -1.5])
def test_upwind3_exact_for_cubics_and_third_order(v):
    """Away from the periodic seam the four-point difference reproduces the
    derivative of any cubic exactly, and on a smooth periodic function its
    error falls as dx^3."""
    from oracle.operators import upwind3
    n = 32
    dx = 1.0 / n
    x = np.arange(n) * dx
    X = np.tile(x, (5, 1))
    for coeffs in ([1.0, 0, 0, 0], [0.3, -2.0, 0, 0], [0.5, 1.0, -3.0, 0], [2.0, -1.0, 0.5, 4.0]):
        f = np.polyval(coeffs[::-1], X)
        df = np.polyval(np.polyder(np.array(coeffs[::-1])), X)
        got = upwind3(f, v, 0.0, dx, 1.0)
        assert np.max(np.abs(got[:, 3:-3] - v * df[:, 3:-3])) <= 1e-9 * max(1.0, np.max(np.abs(v * df)))
    errs = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        X = np.tile(np.arange(n) * dx, (3, 1))
        f = np.sin(2 * np.pi * X)
        got = upwind3(f, v, 0.0, dx, 1.0)
        errs.append(np.max(np.abs(got - v * 2 * np.pi * np.cos(2 * np.pi * X))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.9 < r < 3.1 for r in rates), rates


@pytest.mark.parametrize("D,vx,vy,n", [(1.0, 8.0, 8.0, 8), (0.3, -20.0, 5.0, 8), (0.01, 3.0, -2.0, 6)])
def test_diffadv3_cfl_bound_covers_spectrum(D, vx, vy, n):
    from oracle.operators import diffadv3_apply
    from paper_2310_08344_amd.workloads import diffadv3_cfl_step
    A = dense_matrix(lambda y: diffadv3_apply(y, D, vx, vy, 1 / n, 1 / n), n, n)
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    # the Gershgorin bound equals the largest row sum of moduli of A
    gersh = np.max(np.sum(np.abs(A), axis=1))
    assert abs(2.0 / diffadv3_cfl_step(D, vx, vy, 1 / n, 1 / n) - gersh) <= 1e-10 * gersh
    assert rho <= gersh * (1 + 1e-12)


def test_diffadv3_conserves_sum():
    from oracle.operators import diffadv3_apply
    rng = np.random.default_rng(5)
    y = rng.standard_normal((12, 16))
    out = diffadv3_apply(y, 1.3, 2.0, -3.0, 1 / 16, 1 / 12)
    assert abs(out.sum()) <= 1e-11 * np.abs(out).sum()
