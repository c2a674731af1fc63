"""Leja points, scalar phi functions and Newton divided differences (oracle).

TEST INFRASTRUCTURE ONLY (see the package header): the HIP library never
imports this module.

Paper passages followed
  * phi functions: Sec. 1, the recursion phi_{l+1}(z) = (phi_l(z) - 1/l!)/z
    with phi_0 = exp.
  * Leja points: Sec. 2.1, the greedy definition (each new point maximises the
    product of distances to the earlier ones over the compact set; the first
    point has maximal modulus), on the interval [-2, 2] that Sec. 2.1 names.
  * Newton coefficients: Sec. 2.1, Eq. (2): the interpolant of
    f(xi) = phi_l(c + gamma*xi) in Newton form at the Leja points; its
    coefficients d_j are the divided differences f[xi_0, ..., xi_j].

Readings (paper silent or ambiguous)
  * Ties (the first point is +2 or -2; the fourth is +-2/sqrt(3)) go to the
    larger point, so xi_0 = 2 and z = h*(c + 2*gamma) = 0 is a node.
  * The time step enters the interpolated function, f(xi) = sigma *
    phi_l(alpha*h*(c + gamma*xi)), with c, gamma describing the spectrum of A
    (not of hA); alpha scales the argument and sigma is a prefactor, both 1
    unless an integrator stage asks otherwise.
  * Divided differences are formed by the standard table recurrence in 50
    significant digits and rounded to FP64 once.
"""
from __future__ import annotations

import functools
import math

import mpmath as mp
import numpy as np

DPS = 50


# --------------------------------------------------------------------------
# scalar phi functions (Sec. 1)
# --------------------------------------------------------------------------

def phi_mp(l: int, z) -> mp.mpf:
    """phi_l(z) for real z, in the current mpmath precision.

    |z| >= 1: phi_0 = exp(z) followed by l steps of the Sec. 1 recursion.
    0 < |z| < 1: the recursion's removable-singularity form, the Taylor
    series sum_k z^k/(k+l)!, summed until terms fall below the precision.
    z = 0: phi_l(0) = 1/l!.
    """
    z = mp.mpf(z)
    if z == 0:
        return 1 / mp.factorial(l)
    if abs(z) >= 1:
        val = mp.exp(z)
        for k in range(l):
            val = (val - 1 / mp.factorial(k)) / z
        return val
    term = 1 / mp.factorial(l)
    total = mp.mpf(0)
    k = 0
    eps = mp.mpf(10) ** (-(mp.mp.dps + 5))
    while abs(term) > eps:
        total += term
        k += 1
        term = term * z / (k + l)
    return total


def phi_complex(l: int, z: np.ndarray) -> np.ndarray:
    """phi_l(z) elementwise for complex FP64 arrays (used by the FFT
    reference).  Series sum_k z^k/(k+l)! for |z| < 1, else the Sec. 1
    recursion from exp(z)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    acc = np.zeros_like(zs)
    for k in range(30, -1, -1):          # Horner form of the truncated series
        acc = acc * zs + 1.0 / math.factorial(k + l)
    out[small] = acc
    zb = z[~small]
    val = np.exp(zb)
    for k in range(l):
        val = (val - 1.0 / math.factorial(k)) / zb
    out[~small] = val
    return out


# --------------------------------------------------------------------------
# Leja points on [-2, 2] (Sec. 2.1)
# --------------------------------------------------------------------------

def _log_prod(x: float, pts) -> float:
    return float(sum(math.log(abs(x - p)) for p in pts))


def _bisect_gap(a: float, b: float, pts: np.ndarray) -> float:
    """Maximiser of sum_k log|x - pts_k| inside the gap (a, b) that contains
    no point.  The sum is concave there, so its derivative
    sum_k 1/(x - pts_k) falls from +inf to -inf; bisect on its sign."""
    lo, hi = a, b
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        g = float(np.sum(1.0 / (mid - pts)))
        if g == 0.0:
            return mid
        if g > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@functools.lru_cache(maxsize=4)
def _leja_cached(M: int) -> tuple:
    # Candidate gaps come from a Chebyshev-spaced grid (dense near +-2 where
    # Leja points cluster); every grid local maximum within a margin of the
    # best is refined exactly by bisection, and the best refined value wins.
    G = 1 << 18
    grid = 2.0 * np.cos(np.pi * (np.arange(G) + 0.5) / G)[::-1]
    logp = np.zeros(G)
    pts: list[float] = []

    def add(x):
        pts.append(x)
        with np.errstate(divide="ignore"):
            logp[:] += np.log(np.abs(grid - x))

    add(2.0)
    while len(pts) < M:
        cands = []
        for e in (2.0, -2.0):            # interval ends not yet taken
            if e not in pts:
                cands.append((_log_prod(e, pts), e))
        P = np.asarray(pts)
        inner = (logp[1:-1] >= logp[:-2]) & (logp[1:-1] >= logp[2:])
        idx = np.nonzero(inner)[0] + 1
        if idx.size:
            vals = logp[idx]
            best = vals.max()
            # grid values sit within ~1e-5 of the true gap maxima (spacing
            # <= 2.4e-5, curvature bounded for M <= 1024): refine every gap
            # whose grid maximum is within 1e-3 of the best one
            keep = idx[vals >= best - 1e-3]
            keep = keep[np.argsort(-logp[keep])][:64]
            srt = np.sort(P)
            for i in keep:
                g = grid[i]
                k = np.searchsorted(srt, g)
                a = srt[k - 1] if k > 0 else -2.0
                b = srt[k] if k < srt.size else 2.0
                x = _bisect_gap(a, b, P)
                cands.append((_log_prod(x, pts), x))
        # largest product wins; (near-)exact ties go to the larger point
        cands.sort(key=lambda t: t[0], reverse=True)
        top = cands[0][0]
        tied = [x for v, x in cands if top - v <= 1e-12 * max(1.0, abs(top))]
        add(max(tied))
    return tuple(pts)


def leja_points(M: int) -> np.ndarray:
    """First M Leja points of [-2, 2] (Sec. 2.1), xi_0 = 2."""
    if M < 1:
        return np.zeros(0)
    return np.array(_leja_cached(int(M)))


# --------------------------------------------------------------------------
# Newton divided differences (Sec. 2.1, Eq. (2))
# --------------------------------------------------------------------------

def divided_differences_mp(xs, fs) -> list:
    """Newton coefficients f[x_0], f[x_0,x_1], ..., f[x_0..x_{M-1}] by the
    standard divided-difference table, in mpmath arithmetic."""
    d = [mp.mpf(f) if not isinstance(f, mp.mpf) else f for f in fs]
    x = [mp.mpf(float(v)) for v in xs]
    M = len(d)
    for j in range(1, M):
        for k in range(M - 1, j - 1, -1):
            d[k] = (d[k] - d[k - 1]) / (x[k] - x[k - j])
    return d


def newton_coeffs(l: int, h: float, c: float, gamma: float, M: int,
                  alpha: float = 1.0, sigma: float = 1.0) -> np.ndarray:
    """FP64 Newton coefficients d_0..d_{M-1} of
    f(xi) = sigma * phi_l(alpha*h*(c + gamma*xi)) at the first M Leja points.

    The FP64 inputs h, c, gamma, alpha, sigma and the FP64 Leja points are
    taken exactly into 50-digit arithmetic; only the final d_j are rounded.
    """
    xi = leja_points(M)
    with mp.workdps(DPS):
        a = mp.mpf(alpha) * mp.mpf(h)
        fs = [mp.mpf(sigma) * phi_mp(l, a * (mp.mpf(c) + mp.mpf(gamma) * mp.mpf(float(x))))
              for x in xi]
        d = divided_differences_mp(xi, fs)
        return np.array([float(v) for v in d])
