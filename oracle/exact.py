"""References for phi_l(hA)v that do not use Leja interpolation (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

* Dense: A is assembled column by column from the stencil on small grids and
  phi_l(hA)v is read off the exponential of the augmented matrix
      [[hA, W], [0, S]],  W = [v, 0, ..., 0] (N x l),  S = l x l upper shift,
  whose last column, rows 0..N-1, is phi_l(hA) v (Al-Mohy and Higham 2011,
  Thm. 2.1; Sidje 1998).  The exponential is scipy's Pade scaling and
  squaring.
* FFT: the periodic constant-coefficient diffusion-advection stencil is
  block-circulant with circulant blocks, hence diagonalised by the 2-D DFT.
  Its symbol is
      lam(tx, ty) = D (2 cos tx - 2)/dx^2 + D (2 cos ty - 2)/dy^2
                    + vx (e^{i tx} - 1)/dx + vy (e^{i ty} - 1)/dy   (v >= 0)
  (v < 0 uses the backward difference, vx (1 - e^{-i tx})/dx), and
  phi_l(hA)v = IFFT(phi_l(h lam) FFT(v)).  This is the Fourier-mode
  eigen-solution of the periodic problem and works at any grid size.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .leja import phi_complex


def dense_matrix(apply_A, ny: int, nx: int) -> np.ndarray:
    """Matrix of a linear map on [ny, nx] arrays (row-major flattening)."""
    N = ny * nx
    A = np.empty((N, N))
    e = np.zeros((ny, nx))
    for col in range(N):
        e.flat[col] = 1.0
        A[:, col] = apply_A(e).ravel()
        e.flat[col] = 0.0
    return A


def phi_dense(A: np.ndarray, v: np.ndarray, l: int, h: float) -> np.ndarray:
    """phi_l(hA) v by the exponential of the augmented matrix."""
    v = np.asarray(v, dtype=np.float64).ravel()
    N = A.shape[0]
    if l == 0:
        return sla.expm(h * A) @ v
    B = np.zeros((N + l, N + l))
    B[:N, :N] = h * A
    B[:N, N] = v
    for i in range(l - 1):
        B[N + i, N + i + 1] = 1.0
    E = sla.expm(B)
    return E[:N, -1]


def diffadv_symbol(ny: int, nx: int, D, vx, vy, dx, dy) -> np.ndarray:
    """Eigenvalue of the stencil for each 2-D Fourier mode, laid out like
    numpy.fft.fft2 output ([ky, kx])."""
    tx = 2.0 * np.pi * np.fft.fftfreq(nx)[None, :]
    ty = 2.0 * np.pi * np.fft.fftfreq(ny)[:, None]
    lam = D * (2.0 * np.cos(tx) - 2.0) / dx**2 + D * (2.0 * np.cos(ty) - 2.0) / dy**2
    if vx >= 0:
        lam = lam + vx * (np.exp(1j * tx) - 1.0) / dx
    else:
        lam = lam + vx * (1.0 - np.exp(-1j * tx)) / dx
    if vy >= 0:
        lam = lam + vy * (np.exp(1j * ty) - 1.0) / dy
    else:
        lam = lam + vy * (1.0 - np.exp(-1j * ty)) / dy
    return lam


def diffadv3_symbol(ny: int, nx: int, D, vx, vy, dx, dy) -> np.ndarray:
    """Eigenvalues of the stencil with the third-order upwind gradient, in the
    numpy.fft.fft2 layout: the Laplacian's symbol plus, per axis with
    t = 2 pi k / n,
        v >= 0:  v (-e^{2it} + 6 e^{it} - 3 - 2 e^{-it}) / (6 d)
        v <  0:  v (2 e^{it} + 3 - 6 e^{-it} + e^{-2it}) / (6 d)."""
    tx = 2.0 * np.pi * np.fft.fftfreq(nx)[None, :]
    ty = 2.0 * np.pi * np.fft.fftfreq(ny)[:, None]
    lam = D * (2.0 * np.cos(tx) - 2.0) / dx**2 + D * (2.0 * np.cos(ty) - 2.0) / dy**2

    def g(t, v, d):
        e = np.exp(1j * t)
        if v >= 0:
            return v * (-e * e + 6.0 * e - 3.0 - 2.0 / e) / (6.0 * d)
        return v * (2.0 * e + 3.0 - 6.0 / e + 1.0 / (e * e)) / (6.0 * d)

    return lam + g(tx, vx, dx) + g(ty, vy, dy)


def linear_step_fft(u: np.ndarray, S, h: float, lam: np.ndarray) -> np.ndarray:
    """Exact solution after a time h of u_t = A u + S (S constant in time, or
    None) for a stencil diagonalised by the 2-D DFT with symbol lam:
    mode by mode, e^{h lam} u_hat + h phi_1(h lam) S_hat."""
    uh = np.fft.fft2(np.asarray(u, dtype=np.float64))
    out = np.exp(h * lam) * uh
    if S is not None:
        out = out + h * phi_complex(1, h * lam) * np.fft.fft2(np.asarray(S, dtype=np.float64))
    return np.fft.ifft2(out).real


def phi_fft(v: np.ndarray, l: int, h: float, D, vx, vy, dx, dy) -> np.ndarray:
    """phi_l(hA) v for the periodic diffusion-advection stencil, via FFT."""
    v = np.asarray(v, dtype=np.float64)
    ny, nx = v.shape
    lam = diffadv_symbol(ny, nx, D, vx, vy, dx, dy)
    out = np.fft.ifft2(phi_complex(l, h * lam) * np.fft.fft2(v))
    return out.real
