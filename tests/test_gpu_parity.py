"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bar: relative L2 error <= 1e-10 in FP64 with equal iteration counts (a
borderline stop decision that flips by one sweep is rerun on the oracle at
the GPU's count and reported); FP32 sweeps within the requested tolerance of
the FP64 oracle.  Sizes span several tiles and ragged tails; the full-size
workloads are checked against the exact Fourier solution and invariants.
"""
import math

import numpy as np
import pytest

from oracle.exact import phi_fft
from oracle.operators import burgers_J, diffadv_apply
from oracle.phi_action import exprb32_step, exprb42_step, leja_phi, power_iteration, ros_euler_step
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import (closed_form_shift, oracle_step_parity, dev, diffadv_setup, host, oracle_parity,
                               rel, say)

pytestmark = pytest.mark.gpu

PARITY = 1e-10


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=1024 * 1024, k_max=4)
    yield c
    c.close()


def _op(prm, prec=B.LX_FP64):
    return B.make_operator(kind=B.LX_OP_DIFFADV2D, nx=prm["nx"], ny=prm["ny"], dx=prm["dx"], dy=prm["dy"],
                           D=prm["D"], vx=prm["vx"], vy=prm["vy"], prec=prec)


def _A(prm):
    return lambda y: diffadv_apply(y, prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])


# ---------------------------------------------------------------------------
# spectral bound
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(64, 64), (200, 136), (97, 75)])
def test_spectrum_matches_oracle(ctx, nx, ny):
    prm, _ = diffadv_setup(nx, ny)
    x0 = np.random.default_rng(5).standard_normal((ny, nx))
    say("spectrum diffadv", nx, ny)
    rho, c, g = ctx.spectrum(_op(prm), x0=dev(x0), iters=20)
    rho_o, _ = power_iteration(_A(prm), x0, 20)
    assert abs(rho - rho_o) <= 1e-12 * rho_o
    assert c == -1.05 * rho / 2 and g == 1.05 * rho / 4


def test_spectrum_burgers_jacobian_matches_oracle(ctx):
    n = 128
    u = W.fourier_modes(n, seed=3)
    x0 = np.random.default_rng(6).standard_normal((n, n))
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=1e-3)
    say("spectrum burgers", n)
    rho, _, _ = ctx.spectrum(op, u=dev(u), x0=dev(x0), iters=20)
    rho_o, _ = power_iteration(lambda w: burgers_J(u, w, 1e-3, 1 / n, 1 / n), x0, 20)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


def test_spectrum_default_start_vector(ctx):
    prm, _ = diffadv_setup(128, 128)
    say("spectrum default x0")
    rho, _, _ = ctx.spectrum(_op(prm), iters=30)
    rho_closed = 2.0 / W.diffadv_cfl_step(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    assert 0.9 * rho_closed <= rho <= rho_closed * (1 + 1e-12)


# ---------------------------------------------------------------------------
# phi actions, diffusion-advection
# ---------------------------------------------------------------------------

def test_exp_workload_64_squared_end_to_end(ctx):
    p, u0 = W.config1()
    op = B.make_operator(p)
    x0 = W.start_vector(p.n)
    say("64^2 exp workload")
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    out = dev(np.zeros_like(u0))
    r = ctx.phi_leja(op, dev(u0), [out], [0], p.h, c, g, rtol=1e-10, max_iters=200)
    assert r.status == B.LX_OK
    A = _A(dict(D=p.D, vx=p.vx, vy=p.vy, dx=p.dx, dy=p.dy))
    _, errs, _ = oracle_parity([host(out)], r.iters,
                               lambda f: leja_phi(A, u0, [(0, 1.0, 1.0)], p.h, c, g, 1e-10, 0.0, 200, f),
                               PARITY)
    exact = phi_fft(u0, 0, p.h, p.D, p.vx, p.vy, p.dx, p.dy)
    assert rel(host(out), exact) <= 1e-9


@pytest.mark.parametrize("nx,ny", [(256, 256), (200, 136), (97, 75), (130, 66), (8, 8), (3, 5)])
def test_vertical_phi123_matches_oracle(ctx, nx, ny):
    prm, h = diffadv_setup(nx, ny, cfl=50.0)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(nx * 1000 + ny).standard_normal((ny, nx))
    outs = [dev(np.zeros((ny, nx))) for _ in range(3)]
    say("phi123", nx, ny)
    r = ctx.phi_leja(_op(prm), dev(v), outs, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK
    spec = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)


def test_vertical_outputs_equal_single_runs_bitwise(ctx):
    prm, h = diffadv_setup(192, 160)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = dev(np.random.default_rng(3).standard_normal((160, 192)))
    outs = [dev(np.zeros((160, 192))) for _ in range(3)]
    say("vertical vs single")
    r = ctx.phi_leja(_op(prm), v, outs, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    for k, l in enumerate([1, 2, 3]):
        o = dev(np.zeros((160, 192)))
        rk = ctx.phi_leja(_op(prm), v, [o], [l], h, c, g, rtol=1e-8, max_iters=200)
        assert rk.iters[0] == r.iters[k]
        assert np.array_equal(host(o), host(outs[k]))


def test_alpha_sigma_and_negative_velocity(ctx):
    prm, h = diffadv_setup(144, 96, D=0.3, vx=-20.0, vy=35.0, cfl=20.0)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(9).standard_normal((96, 144))
    outs = [dev(np.zeros((96, 144))) for _ in range(2)]
    spec = [(1, 0.75, 0.75), (0, 0.5, -2.0)]
    say("alpha sigma")
    r = ctx.phi_leja(_op(prm), dev(v), outs, [1, 0], h, c, g, alphas=[0.75, 0.5], sigmas=[0.75, -2.0],
                     rtol=1e-9, atol=1e-12, max_iters=200)
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-9, 1e-12, 200, f), PARITY)


def test_phi123_1024_squared_workload(ctx):
    p, v = W.config2(n=1024)
    op = B.make_operator(p)
    x0 = W.start_vector(p.n)
    say("1024^2 phi123 workload")
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    rho_o, _ = power_iteration(_A(dict(D=p.D, vx=p.vx, vy=p.vy, dx=p.dx, dy=p.dy)), x0, 20)
    assert abs(rho - rho_o) <= 1e-12 * rho_o
    outs = [dev(np.zeros_like(v)) for _ in range(3)]
    r = ctx.phi_leja(op, dev(v), outs, [1, 2, 3], p.h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK
    A = _A(dict(D=p.D, vx=p.vx, vy=p.vy, dx=p.dx, dy=p.dy))
    spec = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(A, v, spec, p.h, c, g, 1e-8, 0.0, 200, f), PARITY)


# ---------------------------------------------------------------------------
# Burgers Jacobian and EXPRB42
# ---------------------------------------------------------------------------

def test_burgers_jacobian_phi_matches_oracle(ctx):
    n = 160
    u = W.fourier_modes(n, seed=3)
    nu = 1e-3
    h = 10.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(u))), 1 / n, 1 / n)
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=nu)
    x0 = np.random.default_rng(7).standard_normal((n, n))
    say("burgers phi", n)
    rho, c, g = ctx.spectrum(op, u=dev(u), x0=dev(x0), iters=20)
    v = np.random.default_rng(8).standard_normal((n, n))
    outs = [dev(np.zeros((n, n))) for _ in range(3)]
    r = ctx.phi_leja(op, dev(v), outs, [1, 1, 3], h, c, g, u=dev(u), alphas=[0.75, 1.0, 1.0],
                     sigmas=[0.75, 1.0, 32 / 9], rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK
    J = lambda w: burgers_J(u, w, nu, 1 / n, 1 / n)
    spec = [(1, 0.75, 0.75), (1, 1.0, 1.0), (3, 1.0, 32 / 9)]
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(J, v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)


@pytest.mark.parametrize("n", [128, 250])
def test_exprb42_step_matches_oracle(ctx, n):
    p, u0 = W.config3(n=n)
    op = B.make_operator(p)
    x0 = np.random.default_rng(11).standard_normal((n, n))
    say("exprb42", n)
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(x0), iters=20)
    out = dev(np.zeros_like(u0))
    r = ctx.exprb_step(op, dev(u0), out, p.h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK
    assert len(r.iters) == 3
    oracle_step_parity(host(out), r.iters,
                       lambda f: exprb42_step(u0, p.nu, p.dx, p.dy, p.h, c, g, 1e-8, 0.0, 200, force_iters=f), PARITY)


STEPS = {"ros_euler": (B.LX_ROS_EULER, ros_euler_step), "exprb32": (B.LX_EXPRB32, exprb32_step),
         "exprb42": (B.LX_EXPRB42, exprb42_step)}


@pytest.mark.parametrize("depth", [4, 2, 1])
@pytest.mark.parametrize("scheme", sorted(STEPS))
@pytest.mark.parametrize("n", [128, 250])
def test_integrator_steps_match_oracle(ctx, scheme, n, depth):
    """Each scheme's step, one or two Leja iterations per launch, against the
    oracle's step (the stages, the sum order and the stop rule of every phi
    pass as in the oracle), at cell Peclet number 2 and h = 10 x CFL."""
    code, oracle_step = STEPS[scheme]
    u0 = W.fourier_modes(n, seed=3)
    nu = float(np.max(np.abs(u0))) / n / 2.0
    h = 10.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(u0))), 1 / n, 1 / n)
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=nu)
    x0 = np.random.default_rng(11).standard_normal((n, n))
    say("integrator", scheme, n, "depth", depth)
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(x0), iters=20)
    out = dev(np.zeros_like(u0))
    ctx.set_depth(depth)
    try:
        r = ctx.exprb_step(op, dev(u0), out, h, c, g, rtol=1e-8, max_iters=200, scheme=code)
    finally:
        ctx.set_depth(0)
    assert r.status == B.LX_OK and r.stats["depth"] == depth
    ref, _, _ = oracle_step_parity(
        host(out), r.iters, lambda f: oracle_step(u0, nu, 1 / n, 1 / n, h, c, g, 1e-8, 0.0, 200, force_iters=f),
        PARITY)
    if scheme == "exprb32":
        # the embedded estimate, through the out-parameter and the stats
        assert abs(r.err[0] - ref.stages["error"]) <= 1e-9 * ref.stages["error"]
        assert r.stats["step_err"] == r.err[0]
    else:
        assert r.err[0] == 0.0


@pytest.mark.parametrize("n", [96, 130])
def test_exprb32_embedded_solution_out_parameter(ctx, n):
    """d_u_low receives the embedded second-order solution a = u + h phi_1(hJ)F(u)
    and err its distance from u+ (rms), both against the oracle's step; the
    other schemes reject d_u_low."""
    u0 = W.fourier_modes(n, seed=5)
    nu = float(np.max(np.abs(u0))) / n / 2.0
    h = 10.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(u0))), 1 / n, 1 / n)
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=nu)
    say("exprb32 embedded", n)
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(W.start_vector(n)), iters=20)
    out, low = dev(np.zeros_like(u0)), dev(np.zeros_like(u0))
    r = ctx.exprb_step(op, dev(u0), out, h, c, g, rtol=1e-8, max_iters=200, scheme=B.LX_EXPRB32, u_low=low)
    assert r.status == B.LX_OK
    ref, _, _ = oracle_step_parity(
        host(out), r.iters, lambda f: exprb32_step(u0, nu, 1 / n, 1 / n, h, c, g, 1e-8, 0.0, 200, force_iters=f),
        PARITY)
    assert rel(host(low), ref.stages["a"]) <= PARITY
    assert abs(r.err[0] - ref.stages["error"]) <= 1e-9 * ref.stages["error"]
    assert abs(r.err[0] - float(np.linalg.norm(host(out) - host(low))) / n) <= 1e-9 * r.err[0]
    for code in (B.LX_EXPRB42, B.LX_ROS_EULER):
        assert ctx.exprb_step(op, dev(u0), out, h, c, g, scheme=code, u_low=low,
                              raise_on_error=False).status == B.LX_EINVAL
    assert ctx.exprb_step(op, dev(u0), out, h, c, g, scheme=B.LX_EXPRB32, u_low=out,
                          raise_on_error=False).status == B.LX_EINVAL


# ---------------------------------------------------------------------------
# FP32 sweeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("switch", [1e4, 0.0])
def test_fp32_sweeps_against_fp64_oracle(ctx, switch):
    prm, h = diffadv_setup(256, 192)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(21).standard_normal((192, 256))
    outs = [dev(np.zeros((192, 256))) for _ in range(3)]
    say("fp32 sweeps", switch)
    r = ctx.phi_leja(_op(prm, prec=B.LX_FP32_SWEEP), dev(v), outs, [1, 2, 3], h, c, g, rtol=1e-8,
                     max_iters=200, fp32_switch=switch)
    assert r.status == B.LX_OK
    assert r.stats["n_fp32"] > 0
    ref = leja_phi(_A(prm), v, [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)], h, c, g, 1e-8, 0.0, 200)
    errs = [rel(host(o), q) for o, q in zip(outs, ref.p)]
    say("fp32 sweep errors vs fp64 oracle", errs, "sweeps", r.stats["n_apply"], "fp32", r.stats["n_fp32"])
    if switch > 0:
        assert max(errs) <= 1e-8
    else:
        assert max(errs) <= 1e-5


def test_fp32_exprb42_against_fp64_oracle(ctx):
    n = 192
    p, u0 = W.config3(n=n)
    op = B.make_operator(p)
    op32 = B.make_operator(p)
    op32.prec = B.LX_FP32_SWEEP
    x0 = np.random.default_rng(12).standard_normal((n, n))
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(x0), iters=20)
    out = dev(np.zeros_like(u0))
    say("fp32 exprb42", n)
    r = ctx.exprb_step(op32, dev(u0), out, p.h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK and r.stats["n_fp32"] > 0
    ref = exprb42_step(u0, p.nu, p.dx, p.dy, p.h, c, g, 1e-8, 0.0, 200)
    err = rel(host(out) - u0, ref.u_next - u0)
    say("fp32 exprb42 error of the update", err)
    assert err <= 1e-7


# ---------------------------------------------------------------------------
# edge cases and error paths
# ---------------------------------------------------------------------------

def test_zero_input_converges_in_one_sweep(ctx):
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    out = dev(np.full((64, 64), 7.0))
    r = ctx.phi_leja(_op(prm), dev(np.zeros((64, 64))), [out], [1], h, c, g, rtol=1e-8)
    assert r.status == B.LX_OK and r.iters == [1]
    assert not np.any(host(out))


def test_max_iters_gives_notconv_with_last_polynomial(ctx):
    prm, h = diffadv_setup(96, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(4).standard_normal((64, 96))
    out = dev(np.zeros((64, 96)))
    say("notconv")
    r = ctx.phi_leja(_op(prm), dev(v), [out], [0], h, c, g, rtol=1e-12, max_iters=5)
    assert r.status == B.LX_ENOTCONV and r.iters == [5]
    ref = leja_phi(_A(prm), v, [(0, 1.0, 1.0)], h, c, g, 1e-12, 0.0, 5)
    assert ref.status == "notconv"
    assert rel(host(out), ref.p[0]) <= PARITY


def test_nonfinite_input_is_reported(ctx):
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.ones((64, 64))
    v[10, 11] = np.nan
    out = dev(np.zeros((64, 64)))
    r = ctx.phi_leja(_op(prm), dev(v), [out], [0], h, c, g, raise_on_error=False)
    assert r.status == B.LX_ENONFINITE


def test_invalid_arguments_are_rejected(ctx):
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = dev(np.ones((64, 64)))
    o = dev(np.zeros((64, 64)))
    bad = [dict(c=1.0), dict(gamma=0.0), dict(h=-1.0)]
    for kw in bad:
        args = dict(h=h, c=c, gamma=g)
        args.update(kw)
        r = ctx.phi_leja(_op(prm), v, [o], [0], args["h"], args["c"], args["gamma"], raise_on_error=False)
        assert r.status == B.LX_EINVAL, kw
    assert ctx.phi_leja(_op(prm), v, [v], [0], h, c, g, raise_on_error=False).status == B.LX_EINVAL
    assert ctx.phi_leja(_op(prm), v, [o, o], [0, 1], h, c, g, raise_on_error=False).status == B.LX_EINVAL
    assert ctx.phi_leja(_op(prm), v, [o], [9], h, c, g, raise_on_error=False).status == B.LX_EINVAL
    assert ctx.phi_leja(_op(prm), v, [o], [0], h, c, g, max_iters=0, raise_on_error=False).status == B.LX_EINVAL
    big = B.make_operator(kind=B.LX_OP_DIFFADV2D, n=2048, D=1.0)
    assert ctx.phi_leja(big, v, [o], [0], h, c, g, raise_on_error=False).status == B.LX_EINVAL
    burg = B.make_operator(kind=B.LX_OP_BURGERS2D, n=64, nu=1e-3)
    assert ctx.phi_leja(burg, v, [o], [0], h, c, g, raise_on_error=False).status == B.LX_EINVAL
    assert ctx.exprb_step(_op(prm), v, o, h, c, g, raise_on_error=False).status == B.LX_EINVAL
    assert "c" in ctx.last_error() or ctx.last_error()


def test_repeat_calls_are_bitwise_deterministic(ctx):
    prm, h = diffadv_setup(512, 384)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = dev(np.random.default_rng(13).standard_normal((384, 512)))
    a = [dev(np.zeros((384, 512))) for _ in range(2)]
    b = [dev(np.zeros((384, 512))) for _ in range(2)]
    say("determinism")
    ra = ctx.phi_leja(_op(prm), v, a, [0, 2], h, c, g, rtol=1e-8)
    rb = ctx.phi_leja(_op(prm), v, b, [0, 2], h, c, g, rtol=1e-8)
    assert ra.iters == rb.iters and ra.err == rb.err
    for x, y in zip(a, b):
        assert np.array_equal(host(x), host(y))


# ---------------------------------------------------------------------------
# launch shapes: every shape the tuner can pick gives the same answer
# ---------------------------------------------------------------------------

TILES = [(64, 4, 1, 2), (64, 4, 8, 2), (32, 8, 2, 2), (16, 16, 4, 2), (8, 32, 1, 2), (4, 64, 8, 2),
         (64, 4, 4, 1), (32, 8, 8, 1), (4, 64, 1, 1)]


@pytest.mark.parametrize("tile", TILES)
def test_every_launch_shape_matches_oracle(ctx, tile):
    prm, h = diffadv_setup(200, 136)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(31).standard_normal((136, 200))
    outs = [dev(np.zeros((136, 200))) for _ in range(3)]
    say("forced tile", tile)
    ctx.set_tile(*tile)
    ctx.set_depth(1)
    try:
        r = ctx.phi_leja(_op(prm), dev(v), outs, [0, 1, 3], h, c, g, rtol=1e-8, max_iters=200)
        n = 120
        u = W.fourier_modes(n, seed=5)
        op_b = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=n, ny=90, dx=1 / n, dy=1 / 90, nu=2e-3)
        ub = u[:90, :]
        x0 = np.random.default_rng(1).standard_normal((90, n))
        rho, cb, gb = ctx.spectrum(op_b, u=dev(ub), x0=dev(x0), iters=20)
        vb = np.random.default_rng(2).standard_normal((90, n))
        ob = dev(np.zeros((90, n)))
        hb = 5.0 * W.burgers_cfl_step(2e-3, float(np.max(np.abs(ub))), 1 / n, 1 / 90)
        rb = ctx.phi_leja(op_b, dev(vb), [ob], [1], hb, cb, gb, u=dev(ub), rtol=1e-8, max_iters=200)
    finally:
        ctx.set_tile(0, 0, 0, 0)
        ctx.set_depth(0)
    assert r.stats["depth"] == 1 and rb.stats["depth"] == 1
    spec = [(0, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)
    rho_o, _ = power_iteration(lambda w: burgers_J(ub, w, 2e-3, 1 / n, 1 / 90), x0, 20)
    assert abs(rho - rho_o) <= 1e-12 * rho_o
    oracle_parity([host(ob)], rb.iters,
                  lambda f: leja_phi(lambda w: burgers_J(ub, w, 2e-3, 1 / n, 1 / 90), vb, [(1, 1.0, 1.0)],
                                     hb, cb, gb, 1e-8, 0.0, 200, f), PARITY)


# ---------------------------------------------------------------------------
# two iterations per launch: the oracle, and one iteration per launch
# ---------------------------------------------------------------------------

PAIR_SHAPES = [(8, 0), (16, 0), (32, 0), (16, 8), (8, 24), (32, 16)]


def _solve_depth(ctx, depth, th, nb, op, v, ls, h, c, g, u=None, **kw):
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, th, nb)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, u=None if u is None else dev(u), **kw)
    finally:
        ctx.set_depth(0)
    return r, [host(o) for o in outs]


@pytest.mark.parametrize("th,nb", PAIR_SHAPES)
def test_two_iteration_launches_match_oracle(ctx, th, nb):
    """Ragged tiles in both directions (200 = 128 + 72 columns, 136 rows),
    phi_0, phi_1, phi_3 from one basis; a Burgers Jacobian with u staged
    beside y; against the oracle and against one iteration per launch."""
    prm, h = diffadv_setup(200, 136)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(31).standard_normal((136, 200))
    say("pair shape", th, nb)
    r2, o2 = _solve_depth(ctx, 2, th, nb, _op(prm), v, [0, 1, 3], h, c, g, rtol=1e-8, max_iters=200)
    r1, o1 = _solve_depth(ctx, 1, 0, 0, _op(prm), v, [0, 1, 3], h, c, g, rtol=1e-8, max_iters=200)
    assert r2.stats["depth"] == 2 and r1.stats["depth"] == 1
    spec = [(0, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o2, r2.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)
    if r2.iters == r1.iters:
        assert max(rel(a, b) for a, b in zip(o2, o1)) <= 1e-13
    n = 120
    ub = W.fourier_modes(n, seed=5)[:90, :]
    op_b = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=n, ny=90, dx=1 / n, dy=1 / 90, nu=2e-3)
    vb = np.random.default_rng(2).standard_normal((90, n))
    hb = 5.0 * W.burgers_cfl_step(2e-3, float(np.max(np.abs(ub))), 1 / n, 1 / 90)
    rho = 2.0 / W.burgers_cfl_step(2e-3, float(np.max(np.abs(ub))), 1 / n, 1 / 90)
    cb, gb = -1.05 * rho / 2.0, 1.05 * rho / 4.0
    rb, ob = _solve_depth(ctx, 2, th, nb, op_b, vb, [1, 2], hb, cb, gb, u=ub, rtol=1e-8, max_iters=200)
    assert rb.stats["depth"] == 2
    Ab = lambda w: burgers_J(ub, w, 2e-3, 1 / n, 1 / 90)
    oracle_parity(ob, rb.iters, lambda f: leja_phi(Ab, vb, [(1, 1.0, 1.0), (2, 1.0, 1.0)], hb, cb, gb, 1e-8, 0.0,
                                                    200, f), PARITY)


@pytest.mark.parametrize("nx,ny", [(6, 5), (4, 3), (130, 7), (256, 40)])
def test_two_iteration_launches_small_and_odd_grids(ctx, nx, ny):
    """Grids narrower than a tile (indices wrap several times), an odd
    number of rows, a single partial tile row."""
    prm, h = diffadv_setup(nx, ny, cfl=20.0)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(nx * 100 + ny).standard_normal((ny, nx))
    say("pair small grid", nx, ny)
    r, o = _solve_depth(ctx, 2, 16, 0, _op(prm), v, [0, 2, 1, 3], h, c, g, rtol=1e-9, max_iters=300)
    assert r.stats["depth"] == 2
    spec = [(0, 1.0, 1.0), (2, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)


@pytest.mark.parametrize("max_iters", [1, 2, 5, 6])
def test_two_iteration_launches_at_max_iters(ctx, max_iters):
    """An odd and an even budget end on the first and on the second test of
    a launch (the even one with a deferred last term)."""
    prm, h = diffadv_setup(96, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(4).standard_normal((64, 96))
    say("pair notconv", max_iters)
    r, o = _solve_depth(ctx, 2, 16, 0, _op(prm), v, [0], h, c, g, rtol=1e-12, max_iters=max_iters,
                        raise_on_error=False)
    assert r.status == B.LX_ENOTCONV and r.iters == [max_iters]
    ref = leja_phi(_A(prm), v, [(0, 1.0, 1.0)], h, c, g, 1e-12, 0.0, max_iters)
    assert rel(o[0], ref.p[0]) <= PARITY
    F = (max_iters + 1) // 2
    assert r.stats["n_launch"] == F + (1 if max_iters % 2 == 0 else 0)
    assert r.stats["n_apply"] == 2 * F


def test_two_iteration_exprb42_matches_one_iteration(ctx):
    n = 128
    u0 = W.fourier_modes(n, seed=9)
    nu = 1e-3
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=nu)
    h = 10.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(u0))), 1 / n, 1 / n)
    rho, c, g = ctx.spectrum(op, u=dev(u0), iters=20)
    outs = {}
    for depth in (2, 1):
        o = dev(np.zeros((n, n)))
        ctx.set_depth(depth)
        try:
            say("exprb42 depth", depth)
            r = ctx.exprb_step(op, dev(u0), o, h, c, g, rtol=1e-8, max_iters=300)
        finally:
            ctx.set_depth(0)
        assert r.status == B.LX_OK and r.stats["depth"] == depth
        outs[depth] = (host(o), r.iters)
    oracle_step_parity(outs[2][0], outs[2][1],
                       lambda f: exprb42_step(u0, nu, 1 / n, 1 / n, h, c, g, 1e-8, 0.0, 300, force_iters=f), PARITY)
    if outs[2][1] == outs[1][1]:
        assert rel(outs[2][0] - u0, outs[1][0] - u0) <= 1e-12


def test_tune_then_solve(ctx):
    prm, h = diffadv_setup(384, 256)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    say("tune 384x256")
    rows = ctx.tune(_op(prm), K=2, sweeps=3)
    assert len(rows) >= 4 and all(r[5] > 0 for r in rows)
    # one iteration per launch, two, windows of three, four and six on LDS
    # tiles, and register-marching windows of four, six and eight (100 + D)
    assert {r[0] for r in rows} == {1, 2, 3, 4, 6, 104, 106, 108}
    v = np.random.default_rng(41).standard_normal((256, 384))
    outs = [dev(np.zeros((256, 384))) for _ in range(2)]
    r = ctx.phi_leja(_op(prm), dev(v), outs, [1, 2], h, c, g, rtol=1e-8, max_iters=200)
    fastest = min(rows, key=lambda q: q[6])
    assert r.stats["depth"] == fastest[0] % 100
    spec = [(1, 1.0, 1.0), (2, 1.0, 1.0)]
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)


def test_bandwidth_probe_reports_plausible_rates(ctx):
    for kind in (0, 1):
        gbs = ctx.bandwidth_probe(kind, 1 << 22, reps=5)
        assert 50.0 < gbs < 20000.0
