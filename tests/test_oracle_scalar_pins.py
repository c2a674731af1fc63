"""Pins of the oracle's scalar parts against facts fixed outside the oracle.

* phi_l: the integral representation phi_l(z) = int_0^1 e^{(1-t) z}
  t^{l-1}/(l-1)! dt (l >= 1), phi_0 = exp, phi_l(0) = 1/l! (Sec. 1 defines
  phi_l by its recursion; the integral form is the textbook equivalent).
* Leja points: the closed-form first points and a brute-force check of the
  greedy maximum property of Sec. 2.1 on a fine grid.
* Divided differences: exact values for a polynomial, and the Opitz identity
  (the first column of f(Z), Z lower bidiagonal with the nodes on the
  diagonal and ones below it, holds the Newton divided differences), with
  f(Z) from mpmath's matrix exponential of an augmented matrix.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.leja import (divided_differences_mp, leja_points, newton_coeffs,
                         phi_complex, phi_mp)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("z", [-80.0, -26.25, -3.0, -1.0, -0.5, -1e-3, 0.0, 1e-7, 0.7, 2.5])
def test_phi_mp_matches_integral_form(l, z):
    with mp.workdps(40):
        got = phi_mp(l, z)
        if l == 0:
            ref = mp.exp(z)
        elif z == 0.0:
            ref = 1 / mp.factorial(l)
        else:
            ref = mp.quad(lambda t: mp.exp((1 - t) * z) * t ** (l - 1) / mp.factorial(l - 1), [0, 1])
        assert abs(got - ref) <= mp.mpf(10) ** -30 * max(1, abs(ref))


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_phi_complex_matches_integral_form(l):
    zs = np.array([-3 + 2j, 0.3 - 0.4j, -0.05 + 0.9j, -100 + 50j, -7.5 - 0.1j, 1e-9 + 0j, -1.0 + 0j])
    got = phi_complex(l, zs)
    with mp.workdps(30):
        for z, g in zip(zs, got):
            zc = mp.mpc(z.real, z.imag)
            if l == 0:
                ref = mp.exp(zc)
            else:
                ref = mp.quad(lambda t: mp.exp((1 - t) * zc) * t ** (l - 1) / mp.factorial(l - 1), [0, 1])
            ref = complex(ref)
            assert abs(g - ref) <= 1e-14 * max(1.0, abs(ref)), (l, z, g, ref)


def test_leja_first_points_closed_form():
    x = leja_points(4)
    assert x[0] == 2.0 and x[1] == -2.0 and x[2] == 0.0
    assert abs(x[3] - 2.0 / math.sqrt(3.0)) <= 4e-16


def test_leja_greedy_max_property_brute_force():
    x = leja_points(48)
    g = np.linspace(-2.0, 2.0, 2_000_001)
    logp = np.zeros_like(g)
    with np.errstate(divide="ignore"):
        for j in range(1, 48):
            logp += np.log(np.abs(g - x[j - 1]))
            val = float(np.sum(np.log(np.abs(x[j] - x[:j]))))
            best = float(np.max(logp))
            # no grid point beats the chosen point, and the chosen point is
            # at least as good as the best grid point up to grid resolution
            assert val >= best - 1e-7 * max(1.0, abs(best)), j
            assert val <= best + 1e-3, j


def test_leja_points_distinct_and_inside():
    x = leja_points(512)
    assert len(np.unique(x)) == 512
    assert np.all(np.abs(x) <= 2.0)
    # Leja points of an interval equidistribute like Chebyshev points: the
    # first 512 fill [-2, 2] with no gap wider than a few times pi*2/512
    s = np.sort(x)
    assert np.max(np.diff(s)) < 4.0 * math.pi * 2.0 / 512


def test_divided_differences_of_a_polynomial_are_exact():
    x = leja_points(10)
    with mp.workdps(50):
        f = [mp.mpf(float(xx)) ** 3 - 2 * mp.mpf(float(xx)) + 1 for xx in x]
        d = divided_differences_mp(x, f)
        # Newton form at nodes x_0..: leading coefficient 1 at order 3,
        # zero beyond; the order-0 value is f(x_0)
        assert abs(d[0] - f[0]) < mp.mpf(10) ** -45
        assert abs(d[3] - 1) < mp.mpf(10) ** -40
        for j in range(4, 10):
            assert abs(d[j]) < mp.mpf(10) ** -38


def _opitz_phi(l, a, b, nodes):
    """First column of phi_l(a*Z + b*I) for the bidiagonal Z of the nodes,
    from one matrix exponential of an augmented matrix (mpmath)."""
    M = len(nodes)
    X = mp.zeros(M + l, M + l)
    for i in range(M):
        X[i, i] = a * mp.mpf(float(nodes[i])) + b
        if i > 0:
            X[i, i - 1] = a
    if l == 0:
        E = mp.expm(X[:M, :M])
        return [E[i, 0] for i in range(M)]
    X[0, M] = 1                 # W = e_0 (the starting vector) in column M
    for i in range(l - 1):
        X[M + i, M + i + 1] = 1
    E = mp.expm(X)
    return [E[i, M + l - 1] for i in range(M)]


@pytest.mark.parametrize("l,hgamma", [(0, 2.0), (0, 26.25), (1, 26.25), (3, 10.0)])
def test_newton_coeffs_match_opitz_matrix_function(l, hgamma):
    # f(xi) = phi_l(h (c + gamma xi)) with c = -2 gamma, i.e.
    # phi_l(hgamma*xi - 2*hgamma): the divided differences over the nodes are
    # the first column of phi_l(hgamma*Z - 2*hgamma*I)
    M = 28
    h, gamma = 1.0, hgamma
    c = -2.0 * gamma
    d = newton_coeffs(l, h, c, gamma, M)
    x = leja_points(M)
    with mp.workdps(60):
        ref = _opitz_phi(l, mp.mpf(hgamma), mp.mpf(-2 * hgamma), x)
    for j in range(M):
        r = float(ref[j])
        assert abs(d[j] - r) <= 1e-15 * max(abs(r), 1e-300) + 1e-300, (j, d[j], r)


def test_newton_form_interpolates_at_the_nodes():
    M = 40
    h, gamma = 0.5, 30.0
    c = -2.0 * gamma
    d = newton_coeffs(1, h, c, gamma, M)
    x = leja_points(M)
    for t in (x[5], x[17], x[39]):
        # evaluate the Newton form at node t in high precision
        with mp.workdps(40):
            acc, w = mp.mpf(0), mp.mpf(1)
            for j in range(M):
                acc += mp.mpf(d[j]) * w
                w *= mp.mpf(float(t)) - mp.mpf(float(x[j]))
            ref = phi_mp(1, mp.mpf(h) * (mp.mpf(c) + mp.mpf(gamma) * mp.mpf(float(t))))
            assert abs(acc - ref) < 1e-13 * max(1, abs(ref))
