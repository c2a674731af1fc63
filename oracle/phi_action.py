"""Power iteration, the Newton-Leja phi-action loop and EXPRB42 (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper passages followed
  * Spectral bound: Sec. 2 names power iteration for the most dominant
    eigenvalue; Sec. 2.2 (Listing 7) then takes lambda = -1.05 * rho_hat,
    c = lambda/2, gamma = -lambda/4.
  * Leja loop: Sec. 2.1, Eq. (2): p_0 = d_0 y_0 with y_0 = v, then
    y_{m+1} = ((A - c)/gamma - xi_m) y_m and p_{m+1} = p_m + d_{m+1} y_{m+1}.
  * Stop rule: Sec. 2.2 (text with Listing 2): converged when the error
    estimate is at most rtol * ||p|| + atol, with l2 norms divided by sqrt(N).
  * Several outputs from one basis ("vertical" interpolation): Sec. 2.3 and
    Listing 11 (integrator coefficients), Sec. 3 (Problem III).
  * Nonlinear remainder N(w) = f(w) - J(u_n) w: Sec. 2.3 (EXPRB32 text).
  * Linear problems (Sec. 3, Problems I and II): u_{n+1} = exp(h A) u_n
    without a source; with a time-independent source S,
    u_{n+1} = u_n + phi_1(h A) h (A u_n + S).

Readings (paper silent or ambiguous)
  * Power iteration: x_{k+1} = A x_k / ||A x_k||, rho_hat = ||A x_k|| / ||x_k||,
    a fixed number of iterations from a caller-supplied start vector.
  * Error estimate of step m+1: |d_{m+1}| * ||y_{m+1}|| / sqrt(N), tested
    after every iteration; iters counts operator applications.  Each output
    freezes once it passes; the loop ends when all outputs have passed or
    after max_iters applications (status "notconv").  A non-finite norm ends
    the loop with status "nonfinite".
  * Substeps (not in the paper; the Leja loop of Sec. 2.1 loses accuracy
    once alpha*h*gamma is large): with s substeps of tau = alpha*h/s,
    exp(alpha h A) v = exp(tau A)^s v, and for l >= 1 the function
    u(t) = t^l phi_l(tA) v solves u' = A u + t^(l-1)/(l-1)! v, u(0) = 0, so
    by the variation-of-constants formula
        u(t + tau) = e^(tau A) u(t) + sum_{i=1..l} tau^i t^(l-i)/(l-i)! phi_i(tau A) v
    (phi-function time stepping, Niesen and Wright 2012) and
    phi_l(alpha h A) v = u(alpha h) / (alpha h)^l.  phi_1..phi_l(tau A) v come
    from one Newton basis; every substep takes one exp action.
  * Problem II's update is printed without the factor h in front of
    phi_1; the exact solution of u_t = A u + S over a step h has it.
  * EXPRB42 (named in Sec. 1, formula not printed; the published two-stage
    fourth-order exponential Rosenbrock method with c_2 = 3/4):
        U_2     = u + (3/4) h phi_1((3/4) h J) F(u)
        u_{n+1} = u + h phi_1(h J) F(u) + (32/9) h phi_3(h J) [N(U_2) - N(u)]
    with J = J(u) and N(w) = F(w) - J w.  The two phi_1 actions share one
    Newton basis (alpha = 3/4 and 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .leja import leja_points, newton_coeffs
from .operators import burgers_F, burgers_J


def _rms(x) -> float:
    """l2 norm divided by sqrt(N) (Sec. 2.2)."""
    return float(np.linalg.norm(x.ravel()) / math.sqrt(x.size))


# --------------------------------------------------------------------------
# spectral bound
# --------------------------------------------------------------------------

def power_iteration(apply_A, x0, iters: int = 20):
    """Returns (rho_hat, history) after ``iters`` applications of A."""
    x = np.array(x0, dtype=np.float64, copy=True)
    hist = []
    for _ in range(iters):
        y = apply_A(x)
        ny = float(np.linalg.norm(y.ravel()))
        hist.append(ny / float(np.linalg.norm(x.ravel())))
        x = y / ny
    return hist[-1], hist


def shift_scale(rho_hat: float, safety: float = 1.05):
    """lambda = -safety * rho_hat, c = lambda/2, gamma = -lambda/4
    (Listing 7): the Leja interval [-2, 2] maps onto [lambda, 0]."""
    lam = -safety * rho_hat
    return lam / 2.0, -lam / 4.0


# --------------------------------------------------------------------------
# Newton-Leja phi actions
# --------------------------------------------------------------------------

@dataclass
class LejaResult:
    p: list            # one output array per requested (l, alpha, sigma)
    iters: list        # operator applications until each output passed
    errs: list         # error estimate of each output at its last step
    status: str        # "ok", "notconv" or "nonfinite"
    n_apply: int       # operator applications made in total


def leja_phi(apply_A, v, outputs, h, c, gamma, rtol, atol, max_iters=500,
             force_iters=None) -> LejaResult:
    """sigma_k * phi_{l_k}(alpha_k h A) v for every (l_k, alpha_k, sigma_k) in
    ``outputs``, by Newton interpolation at the Leja points of [-2, 2].

    ``force_iters`` (int or list) replaces the stop test of an output by a
    fixed iteration count; it exists so that a run can be compared with
    another whose borderline stop decision went the other way.
    """
    v = np.asarray(v, dtype=np.float64)
    K = len(outputs)
    if force_iters is not None and not isinstance(force_iters, (list, tuple)):
        force_iters = [int(force_iters)] * K
    M = max_iters + 1
    xi = leja_points(M)
    d = [newton_coeffs(l, h, c, gamma, M, alpha=a, sigma=s) for (l, a, s) in outputs]

    y = v.copy()
    p = [d[k][0] * v for k in range(K)]
    active = [True] * K
    iters = [max_iters] * K
    errs = [float("nan")] * K
    status = "ok"
    n_apply = 0
    for m in range(max_iters):
        y = (apply_A(y) - c * y) / gamma - xi[m] * y
        n_apply += 1
        ynorm = _rms(y)
        for k in range(K):
            if not active[k]:
                continue
            p[k] = p[k] + d[k][m + 1] * y
            err = abs(d[k][m + 1]) * ynorm
            pnorm = _rms(p[k])
            errs[k] = err
            if not (math.isfinite(err) and math.isfinite(pnorm)):
                status = "nonfinite"
                active[k] = False
                iters[k] = m + 1
                continue
            if force_iters is not None:
                done = (m + 1) >= force_iters[k]
            else:
                done = err <= rtol * pnorm + atol
            if done:
                active[k] = False
                iters[k] = m + 1
        if status == "nonfinite" or not any(active):
            break
    if status == "ok" and any(active):
        status = "notconv"
    return LejaResult(p=p, iters=iters, errs=errs, status=status, n_apply=n_apply)


def substep_count(outputs, h, gamma, hg_max: float = 300.0) -> int:
    """Automatic substep count: the largest alpha*h*gamma split into pieces
    of at most hg_max (reading: 300, half the largest alpha*h*gamma at which
    the plain loop was still seen to converge)."""
    hg = max(a for (_, a, _) in outputs) * h * gamma
    return max(1, math.ceil(hg / hg_max))


def leja_phi_substeps(apply_A, v, outputs, h, c, gamma, rtol, atol, substeps, max_iters=500):
    """sigma_k phi_{l_k}(alpha_k h A) v by ``substeps`` substeps (see the
    module header); every Leja call has its own stop rule.  Returns
    (outputs, iterations per output: the phi_l call it used plus its exp
    calls, status)."""
    v = np.asarray(v, dtype=np.float64)
    s = int(substeps)
    outs, iters, status = [], [], "ok"

    def worst(st):
        nonlocal status
        if st != "ok" and status != "nonfinite":
            status = st

    for (l, a, sg) in outputs:
        H = a * h
        tau = H / s
        if l == 0:
            u, it = v, 0
            for j in range(s):
                r = leja_phi(apply_A, u, [(0, 1.0, sg if j == s - 1 else 1.0)], tau, c, gamma, rtol, atol,
                             max_iters)
                worst(r.status)
                u, it = r.p[0], it + r.iters[0]
            outs.append(u)
            iters.append(it)
            continue
        P = leja_phi(apply_A, v, [(i, 1.0, 1.0) for i in range(1, l + 1)], tau, c, gamma, rtol, atol, max_iters)
        worst(P.status)
        it = P.iters[l - 1]
        u = tau**l * P.p[l - 1]                       # u(tau): t = 0 leaves only i = l
        for j in range(1, s):
            t = j * tau
            r = leja_phi(apply_A, u, [(0, 1.0, 1.0)], tau, c, gamma, rtol, atol, max_iters)
            worst(r.status)
            it += r.iters[0]
            u = r.p[0]
            for i in range(1, l + 1):
                u = u + (tau**i * t ** (l - i) / math.factorial(l - i)) * P.p[i - 1]
        outs.append(sg * u / H**l)
        iters.append(it)
    return outs, iters, status


# --------------------------------------------------------------------------
# linear problems (Problems I and II)
# --------------------------------------------------------------------------

def linear_step(apply_A, u, S, h, c, gamma, rtol, atol, max_iters=500) -> "StepResult":
    """One step of u_t = A u (+ S): the exp action of u when S is None
    (Problem I), else u + phi_1(h A) h (A u + S) (Problem II)."""
    u = np.asarray(u, dtype=np.float64)
    if S is None:
        r = leja_phi(apply_A, u, [(0, 1.0, 1.0)], h, c, gamma, rtol, atol, max_iters)
        return StepResult(u_next=r.p[0], iters=[r.iters[0], 0], status=r.status, stages={})
    w = h * (apply_A(u) + np.asarray(S, dtype=np.float64))
    r = leja_phi(apply_A, w, [(1, 1.0, 1.0)], h, c, gamma, rtol, atol, max_iters)
    return StepResult(u_next=u + r.p[0], iters=[r.iters[0], 0], status=r.status,
                      stages={"rhs": w, "phi1": r.p[0]})


# --------------------------------------------------------------------------
# EXPRB42 for Burgers
# --------------------------------------------------------------------------

@dataclass
class StepResult:
    u_next: np.ndarray
    iters: list        # iterations of every phi action of the step, in the
                       # order the step takes them (see each step function)
    status: str
    stages: dict


def _forced(force_iters, i):
    """Iteration count forced on the i-th phi action of a step, or None.

    A step's actions each have their own stop rule (Sec. 2.2); a borderline
    decision may go the other way in a run whose norms add in another order,
    and the comparison is then made with the oracle forced to that run's
    counts, action by action."""
    return None if force_iters is None else int(force_iters[i])


def ros_euler_step(u, nu, dx, dy, h, c, gamma, rtol, atol, max_iters=500, force_iters=None) -> StepResult:
    """One exponential Rosenbrock-Euler step (Sec. 2.3): the phi_1 action of
    the Jacobian at u on h F(u), added to u.  iters: [phi_1 action];
    ``force_iters`` (the same layout) fixes the counts instead."""
    u = np.asarray(u, dtype=np.float64)
    J = lambda w: burgers_J(u, w, nu, dx, dy)
    hF = h * burgers_F(u, nu, dx, dy)
    r = leja_phi(J, hF, [(1, 1.0, 1.0)], h, c, gamma, rtol, atol, max_iters, _forced(force_iters, 0))
    return StepResult(u_next=u + r.p[0], iters=[r.iters[0]], status=r.status, stages={"phi1": r.p[0]})


def exprb32_step(u, nu, dx, dy, h, c, gamma, rtol, atol, max_iters=500, force_iters=None) -> StepResult:
    """One EXPRB32 step (Sec. 2.3): the Rosenbrock-Euler stage a, then the
    third-order correction 2 phi_3(hJ) h [N(a) - N(u)] with N(w) = F(w) - J w;
    stages["error"] is the rms norm of the correction (the embedded estimate)
    and stages["a"] the embedded second-order solution.  iters: [phi_1,
    phi_3 action]; ``force_iters`` (the same layout) fixes the counts."""
    u = np.asarray(u, dtype=np.float64)
    J = lambda w: burgers_J(u, w, nu, dx, dy)
    F = lambda w: burgers_F(w, nu, dx, dy)
    hF = h * F(u)
    r1 = leja_phi(J, hF, [(1, 1.0, 1.0)], h, c, gamma, rtol, atol, max_iters, _forced(force_iters, 0))
    a = u + r1.p[0]
    Nl = lambda w: F(w) - J(w)
    R = h * (Nl(a) - Nl(u))
    r2 = leja_phi(J, R, [(3, 1.0, 2.0)], h, c, gamma, rtol, atol, max_iters, _forced(force_iters, 1))
    corr = r2.p[0]
    status = r1.status if r1.status != "ok" else r2.status
    return StepResult(u_next=a + corr, iters=[r1.iters[0], r2.iters[0]], status=status,
                      stages={"a": a, "R": R, "correction": corr,
                              "error": float(np.linalg.norm(corr) / math.sqrt(corr.size))})


def exprb42_step(u, nu, dx, dy, h, c, gamma, rtol, atol, max_iters=500, force_iters=None) -> StepResult:
    """One EXPRB42 step of u_t = F(u) (Burgers), Jacobian and remainder as in
    Sec. 2.3; the phi actions use Newton-Leja interpolation.  iters: [the
    (3/4) phi_1((3/4) h J) output and the phi_1(h J) output of the first
    pass (one basis, each with its own stop), the phi_3 action];
    ``force_iters`` (the same layout) fixes the counts."""
    u = np.asarray(u, dtype=np.float64)
    J = lambda w: burgers_J(u, w, nu, dx, dy)
    F = lambda w: burgers_F(w, nu, dx, dy)
    hF = h * F(u)
    f1 = None if force_iters is None else [_forced(force_iters, 0), _forced(force_iters, 1)]
    r1 = leja_phi(J, hF, [(1, 0.75, 0.75), (1, 1.0, 1.0)], h, c, gamma, rtol, atol, max_iters, f1)
    a = r1.p[0]                       # (3/4) h phi_1((3/4) h J) F(u)
    U2 = u + a
    Nl = lambda w: F(w) - J(w)
    R = h * (Nl(U2) - Nl(u))
    r2 = leja_phi(J, R, [(3, 1.0, 32.0 / 9.0)], h, c, gamma, rtol, atol, max_iters, _forced(force_iters, 2))
    u_next = u + r1.p[1] + r2.p[0]
    status = r1.status if r1.status != "ok" else r2.status
    return StepResult(u_next=u_next, iters=[r1.iters[0], r1.iters[1], r2.iters[0]], status=status,
                      stages={"a": a, "phi1": r1.p[1], "R": R, "phi3": r2.p[0]})
