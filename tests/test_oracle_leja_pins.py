"""Pins of the oracle's Newton-Leja loop, power iteration and EXPRB42 against
references that do not use Leja interpolation, and against invariants.

* Dense: phi_l(hA)v from the exponential of the augmented matrix (scipy Pade)
  on 8x8 grids, for the diffusion-advection stencil and the Burgers Jacobian.
* FFT: the exact Fourier-mode solution of the periodic diffusion-advection
  problem, at the 64^2 exp workload and at a 128^2 version of the
  phi_1..phi_3 workload (h = 50 x CFL).
* Invariants: sum conservation (the Newton interpolant takes its value at the
  node xi_0 = 2, i.e. phi_l(0) = 1/l!, on the constant mode), constant data,
  the phi recursion hA phi_{l+1}(hA) v = phi_l(hA) v - v/l! (Sec. 1),
  the semigroup property of exp, linearity in v, and that the "vertical"
  outputs equal separate single-output runs.
* Power iteration: for a normal matrix the norm ratio never exceeds the
  spectral radius and never decreases.
* EXPRB42: fourth order against an independent ODE solution (scipy DOP853).
* Linear problems I and II (Sec. 3) with the third-order upwind gradient:
  one step equals the exact solution of u_t = A u (+ S) over h, computed mode
  by mode as e^{h lam} u_hat + h phi_1(h lam) S_hat.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.exact import dense_matrix, phi_dense, phi_fft
from oracle.operators import burgers_F, burgers_J, diffadv_apply, make_apply
from oracle.phi_action import (exprb32_step, exprb42_step, leja_phi, power_iteration, ros_euler_step,
                               shift_scale)
from paper_2310_08344_amd import workloads as W


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _bounds(apply_A, shape, seed=5, iters=20):
    x0 = np.random.default_rng(seed).standard_normal(shape)
    rho, _ = power_iteration(apply_A, x0, iters)
    return shift_scale(rho)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_leja_matches_dense_expm_diffadv(l):
    n = 8
    D, v = 1.0, 8.0
    h = 10.0 * W.diffadv_cfl_step(D, v, -0.5 * v, 1 / n, 1 / n)
    A_apply = lambda y: diffadv_apply(y, D, v, -0.5 * v, 1 / n, 1 / n)
    c, g = _bounds(A_apply, (n, n))
    rng = np.random.default_rng(11)
    vec = rng.standard_normal((n, n))
    res = leja_phi(A_apply, vec, [(l, 1.0, 1.0)], h, c, g, 1e-10, 0.0, max_iters=200)
    assert res.status == "ok"
    ref = phi_dense(dense_matrix(A_apply, n, n), vec, l, h)
    assert _rel(res.p[0].ravel(), ref) <= 1e-9


@pytest.mark.parametrize("l,alpha", [(1, 0.75), (1, 1.0), (3, 1.0)])
def test_leja_matches_dense_expm_burgers_jacobian(l, alpha):
    n = 8
    u = W.fourier_modes(n, seed=3, kmax=2) + 0.3
    nu = 0.02
    h = 10.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(u))), 1 / n, 1 / n)
    J = lambda w: burgers_J(u, w, nu, 1 / n, 1 / n)
    c, g = _bounds(J, (n, n))
    vec = np.random.default_rng(12).standard_normal((n, n))
    res = leja_phi(J, vec, [(l, alpha, 1.0)], h, c, g, 1e-11, 0.0, max_iters=300)
    assert res.status == "ok"
    ref = phi_dense(dense_matrix(J, n, n), vec, l, alpha * h)
    assert _rel(res.p[0].ravel(), ref) <= 1e-9


@pytest.mark.parametrize("index", [1, 13, 21])
def test_tight_leja_on_learned_burgers_instances_matches_dense_expm(index):
    """The reference the learned-path tests use for Burgers instances (the
    Jacobian is not diagonalised by the FFT): the oracle's loop at rtol 1e-13
    on the closed-form Gershgorin interval, checked here against the dense
    augmented exponential on 24^2 instances of the learned distribution
    (phi_2; cell Peclet numbers 0.3 to 3.4; h from 3.3 to 6.4 x CFL)."""
    prm, u, v = W.learned_instance(index, 720000, (24,))
    A = make_apply(prm, u)
    l = prm.meta["l"]
    rho = 2.0 / W.burgers_cfl_step(prm.nu, float(np.max(np.abs(u))), prm.dx, prm.dy)
    c, g = shift_scale(rho)
    r = leja_phi(A, v, [(l, 1.0, 1.0)], prm.h, c, g, 1e-13, 0.0, 400)
    assert r.status == "ok"
    ex = phi_dense(dense_matrix(A, 24, 24), v, l, prm.h).reshape(24, 24)
    assert _rel(r.p[0], ex) <= 1e-12


def test_leja_matches_fft_on_64_squared_exp_workload():
    p, u0 = W.config1()
    A_apply = make_apply(p)
    c, g = _bounds(A_apply, u0.shape, iters=20)
    res = leja_phi(A_apply, u0, [(0, 1.0, 1.0)], p.h, c, g, 1e-10, 0.0, max_iters=200)
    assert res.status == "ok"
    ref = phi_fft(u0, 0, p.h, p.D, p.vx, p.vy, p.dx, p.dy)
    assert _rel(res.p[0], ref) <= 1e-9


@pytest.mark.slow
def test_leja_matches_fft_on_128_squared_phi123_workload():
    p, vec = W.config2(n=128, seed=1)
    A_apply = make_apply(p)
    c, g = _bounds(A_apply, vec.shape)
    outs = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)]
    res = leja_phi(A_apply, vec, outs, p.h, c, g, 1e-8, 0.0, max_iters=200)
    assert res.status == "ok"
    for k, (l, _, _) in enumerate(outs):
        ref = phi_fft(vec, l, p.h, p.D, p.vx, p.vy, p.dx, p.dy)
        assert _rel(res.p[k], ref) <= 1e-7, (l, _rel(res.p[k], ref))


def _small_problem():
    n = 16
    D, vx, vy = 0.5, 6.0, 3.0
    h = 20.0 * W.diffadv_cfl_step(D, vx, vy, 1 / n, 1 / n)
    A_apply = lambda y: diffadv_apply(y, D, vx, vy, 1 / n, 1 / n)
    c, g = _bounds(A_apply, (n, n))
    return n, h, A_apply, c, g


@pytest.mark.parametrize("l", [0, 1, 3])
def test_sum_invariant_holds_for_the_leja_approximant(l):
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(3).standard_normal((n, n)) + 0.2
    res = leja_phi(A_apply, vec, [(l, 1.0, 1.0)], h, c, g, 1e-6, 0.0, max_iters=200)
    target = vec.sum() / math.factorial(l)
    assert abs(res.p[0].sum() - target) <= 1e-13 * np.abs(vec).sum()


@pytest.mark.parametrize("l", [0, 2])
def test_constant_data_gives_v_over_l_factorial(l):
    n, h, A_apply, c, g = _small_problem()
    vec = np.full((n, n), 2.5)
    res = leja_phi(A_apply, vec, [(l, 1.0, 1.0)], h, c, g, 1e-12, 0.0, max_iters=200)
    assert np.max(np.abs(res.p[0] - vec / math.factorial(l))) <= 1e-13


@pytest.mark.parametrize("l", [0, 1, 2])
def test_phi_recursion_identity(l):
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(4).standard_normal((n, n))
    tol = 1e-11
    r = leja_phi(A_apply, vec, [(l, 1.0, 1.0), (l + 1, 1.0, 1.0)], h, c, g, tol, 0.0, max_iters=200)
    lhs = h * A_apply(r.p[1])
    rhs = r.p[0] - vec / math.factorial(l)
    rho = 2.0 / W.diffadv_cfl_step(0.5, 6.0, 3.0, 1 / n, 1 / n)
    assert np.linalg.norm(lhs - rhs) <= 20 * h * rho * tol * np.linalg.norm(vec)


def test_exp_semigroup():
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(6).standard_normal((n, n))
    tol = 1e-12
    a = leja_phi(A_apply, vec, [(0, 1.0, 1.0)], 0.4 * h, c, g, tol, 0.0, max_iters=200).p[0]
    ab = leja_phi(A_apply, a, [(0, 1.0, 1.0)], 0.6 * h, c, g, tol, 0.0, max_iters=200).p[0]
    full = leja_phi(A_apply, vec, [(0, 1.0, 1.0)], h, c, g, tol, 0.0, max_iters=200).p[0]
    assert _rel(ab, full) <= 1e-10


def test_linearity_in_v():
    n, h, A_apply, c, g = _small_problem()
    rng = np.random.default_rng(7)
    v1, v2 = rng.standard_normal((2, n, n))
    f = lambda vec: leja_phi(A_apply, vec, [(1, 1.0, 1.0)], h, c, g, 0.0, 0.0,
                             max_iters=200, force_iters=60).p[0]
    assert _rel(f(2.0 * v1 - 3.0 * v2), 2.0 * f(v1) - 3.0 * f(v2)) <= 1e-13


def test_vertical_outputs_equal_separate_runs():
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(8).standard_normal((n, n))
    outs = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 0.75, 2.0)]
    joint = leja_phi(A_apply, vec, outs, h, c, g, 1e-9, 0.0, max_iters=200)
    for k, o in enumerate(outs):
        single = leja_phi(A_apply, vec, [o], h, c, g, 1e-9, 0.0, max_iters=200)
        assert single.iters[0] == joint.iters[k]
        assert np.array_equal(single.p[0], joint.p[k])


def test_sigma_and_alpha_scale_as_defined():
    # sigma * phi_l(alpha h A) v equals sigma times the run at step alpha*h
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(9).standard_normal((n, n))
    a = leja_phi(A_apply, vec, [(1, 0.75, 0.75)], h, c, g, 1e-12, 0.0, max_iters=200).p[0]
    b = leja_phi(A_apply, vec, [(1, 1.0, 1.0)], 0.75 * h, c, g, 1e-12, 0.0, max_iters=200).p[0]
    assert _rel(a, 0.75 * b) <= 1e-11


def test_power_iteration_bounds_and_monotone():
    p, u0 = W.config1()
    A_apply = make_apply(p)
    x0 = W.start_vector(p.n)
    rho_hat, hist = power_iteration(A_apply, x0, 20)
    rho = 2.0 / W.diffadv_cfl_step(p.D, p.vx, p.vy, p.dx, p.dy)
    assert rho_hat <= rho * (1 + 1e-12)
    assert all(b >= a * (1 - 1e-13) for a, b in zip(hist, hist[1:]))
    assert rho_hat >= 0.9 * rho


def test_not_converged_and_nonfinite_status():
    n, h, A_apply, c, g = _small_problem()
    vec = np.random.default_rng(10).standard_normal((n, n))
    r = leja_phi(A_apply, vec, [(0, 1.0, 1.0)], h, c, g, 1e-12, 0.0, max_iters=3)
    assert r.status == "notconv" and r.iters == [3] and r.n_apply == 3
    bad = vec.copy()
    bad[3, 4] = np.nan
    r = leja_phi(A_apply, bad, [(0, 1.0, 1.0)], h, c, g, 1e-12, 0.0, max_iters=50)
    assert r.status == "nonfinite" and r.n_apply == 1


def test_zero_vector_converges_in_one_step():
    n, h, A_apply, c, g = _small_problem()
    r = leja_phi(A_apply, np.zeros((n, n)), [(1, 1.0, 1.0)], h, c, g, 1e-8, 0.0, max_iters=50)
    assert r.status == "ok" and r.iters == [1] and not np.any(r.p[0])


def _burgers_orders(step, steps_list, n=16, nu=0.05, T=0.02):
    """Errors of `step` against DOP853 on a smooth Burgers problem, and the
    observed convergence rates when the step is halved."""
    u0 = 1.0 + 0.5 * W.fourier_modes(n, seed=21, n_modes=2, kmax=1)
    dx = 1.0 / n
    sol = solve_ivp(lambda t, y: burgers_F(y.reshape(n, n), nu, dx, dx).ravel(), (0.0, T),
                    u0.ravel(), method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1].reshape(n, n)
    errs, ests = [], []
    for steps in steps_list:
        h = T / steps
        u = u0.copy()
        for _ in range(steps):
            J = lambda w, u=u: burgers_J(u, w, nu, dx, dx)
            x0 = np.random.default_rng(1).standard_normal((n, n))
            rho, _ = power_iteration(J, x0, 30)
            c, g = shift_scale(rho)
            r = step(u, nu, dx, dx, h, c, g, 1e-14, 0.0, max_iters=300)
            if len(ests) < len(errs) + 1 and "error" in r.stages:
                ests.append(r.stages["error"])     # the first step's embedded estimate
            u = r.u_next
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    return errs, rates, ests


@pytest.mark.slow
def test_ros_euler_is_second_order():
    errs, rates, _ = _burgers_orders(ros_euler_step, (4, 8, 16))
    assert min(rates) > 1.8 and max(rates) < 2.3, (errs, rates)


@pytest.mark.slow
def test_exprb32_is_third_order_and_its_estimate_local_third_order():
    errs, rates, ests = _burgers_orders(exprb32_step, (4, 8, 16))
    assert min(rates) > 2.7 and max(rates) < 3.4, (errs, rates)
    # the estimate is the local error of the embedded second-order solution: O(h^3)
    est_rates = [math.log2(a / b) for a, b in zip(ests, ests[1:])]
    assert min(est_rates) > 2.6, (ests, est_rates)


@pytest.mark.slow
def test_exprb42_is_fourth_order():
    n = 16
    nu = 0.05
    u0 = 1.0 + 0.5 * W.fourier_modes(n, seed=21, n_modes=2, kmax=1)
    dx = 1.0 / n
    T = 0.02
    sol = solve_ivp(lambda t, y: burgers_F(y.reshape(n, n), nu, dx, dx).ravel(), (0.0, T),
                    u0.ravel(), method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1].reshape(n, n)
    errs = []
    for steps in (2, 4, 8):
        h = T / steps
        u = u0.copy()
        for _ in range(steps):
            J = lambda w, u=u: burgers_J(u, w, nu, dx, dx)
            x0 = np.random.default_rng(1).standard_normal((n, n))
            rho, _ = power_iteration(J, x0, 30)
            c, g = shift_scale(rho)
            u = exprb42_step(u, nu, dx, dx, h, c, g, 1e-14, 0.0, max_iters=300).u_next
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert errs[-1] < 1e-7
    assert min(rates) > 3.5, (errs, rates)


@pytest.mark.parametrize("n,cfl,source", [(64, 10.0, False), (64, 10.0, True), (50, 100.0, True), (48, 1.0, True)])
def test_linear_step_matches_exact_solution(n, cfl, source):
    from oracle.exact import diffadv3_symbol, linear_step_fft
    from oracle.phi_action import linear_step
    p, u, S = W.paper_linear(n, cfl, source)
    A = make_apply(p)
    c, g = _bounds(A, u.shape)
    r = linear_step(A, u, S, p.h, c, g, 1e-12, 0.0, max_iters=200)
    assert r.status == "ok"
    lam = diffadv3_symbol(n, n, p.D, p.vx, p.vy, p.dx, p.dy)
    assert _rel(r.u_next, linear_step_fft(u, S, p.h, lam)) <= 1e-11


# ---- substeps (phi-function time stepping) --------------------------------

def _paper_fft(n, hg, ls):
    from oracle.exact import diffadv3_symbol
    from oracle.leja import phi_complex
    p, u, _ = W.paper_linear(n, 1.0, False)
    A = make_apply(p)
    c, g = _bounds(A, u.shape)
    h = hg / g
    lam = diffadv3_symbol(n, n, p.D, p.vx, p.vy, p.dx, p.dy)
    ex = [np.fft.ifft2(phi_complex(l, a * h * lam) * np.fft.fft2(u)).real * sg for (l, a, sg) in ls]
    return A, u, h, c, g, ex


@pytest.mark.parametrize("n", [32, 30])
def test_substeps_recover_large_steps(n):
    """At alpha h gamma = 1200 the plain loop diverges; eight substeps give
    the exact Fourier solution for exp and phi_1..phi_3, with alpha and sigma."""
    from oracle.phi_action import leja_phi_substeps, substep_count
    ls = [(0, 1.0, 1.0), (1, 1.0, 1.0), (3, 0.75, 2.0), (2, 1.0, -0.5)]
    A, u, h, c, g, ex = _paper_fft(n, 1200.0, ls)
    plain = leja_phi(A, u, [(0, 1.0, 1.0)], h, c, g, 1e-12, 0.0, 1000)
    assert plain.status != "ok" or _rel(plain.p[0], ex[0]) > 1e-3
    assert substep_count(ls, h, g) == 4
    outs, iters, status = leja_phi_substeps(A, u, ls, h, c, g, 1e-12, 0.0, 8, 500)
    assert status == "ok"
    for o, e in zip(outs, ex):
        assert _rel(o, e) <= 1e-10


def test_one_substep_is_the_plain_loop():
    from oracle.phi_action import leja_phi_substeps
    ls = [(0, 1.0, 1.0), (2, 0.5, 3.0)]
    A, u, h, c, g, ex = _paper_fft(24, 80.0, ls)
    outs, iters, status = leja_phi_substeps(A, u, ls, h, c, g, 1e-12, 0.0, 1, 500)
    r0 = leja_phi(A, u, [ls[0]], h, c, g, 1e-12, 0.0, 500)
    assert np.array_equal(outs[0], r0.p[0]) and iters[0] == r0.iters[0]
    r2 = leja_phi(A, u, [(1, 0.5, 1.0), (2, 0.5, 1.0)], h, c, g, 1e-12, 0.0, 500)
    assert _rel(outs[1], 3.0 * r2.p[1]) <= 1e-14
    for o, e in zip(outs, ex):
        assert _rel(o, e) <= 1e-10
