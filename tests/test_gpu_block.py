"""GPU parity of the speculative-window kernel (three and four Leja
iterations per launch, `leja_block`) against the CPU oracle and against one
iteration per launch, through the C ABI.

Each output must take exactly the terms of the one-iteration loop: the
oracle comparison at 1e-10 with equal iteration counts (a borderline stop
decision flipped by the order of the norm reductions is rerun at the GPU's
count and reported), 1e-13 against depth 1 when the counts agree, stops at
every position inside a window (max_iters 1..9), outputs that stop in
different windows, ragged and tiny grids.
"""
import numpy as np
import pytest

from oracle.exact import phi_fft
from oracle.operators import burgers_J, diffadv_apply
from oracle.phi_action import leja_phi, power_iteration
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import closed_form_shift, dev, diffadv_setup, host, oracle_parity, oracle_step_parity, rel, say

pytestmark = pytest.mark.gpu

PARITY = 1e-10


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=1024 * 1024, k_max=4)
    yield c
    c.close()


def _op(prm):
    return B.make_operator(kind=B.LX_OP_DIFFADV2D, nx=prm["nx"], ny=prm["ny"], dx=prm["dx"], dy=prm["dy"],
                           D=prm["D"], vx=prm["vx"], vy=prm["vy"])


def _A(prm):
    return lambda y: diffadv_apply(y, prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])


def _solve(ctx, depth, th, nb, op, v, ls, h, c, g, **kw):
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, th, nb)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, **kw)
    finally:
        ctx.set_depth(0)
    return r, [host(o) for o in outs]


@pytest.mark.parametrize("depth,th,nb", [(3, 8, 0), (3, 16, 0), (4, 8, 0), (4, 16, 0), (4, 16, 8), (3, 8, 24),
                                         (6, 8, 0), (6, 16, 16)])
def test_windows_match_oracle_and_one_iteration(ctx, depth, th, nb):
    """Ragged tiles both ways (200 = 128 + 72 columns, 136 rows); phi_0,
    phi_1 and phi_3 stop in different windows."""
    prm, h = diffadv_setup(200, 136)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(31).standard_normal((136, 200))
    say("window", depth, th, nb)
    rb, ob = _solve(ctx, depth, th, nb, _op(prm), v, [0, 1, 3], h, c, g, rtol=1e-8, max_iters=200)
    r1, o1 = _solve(ctx, 1, 0, 0, _op(prm), v, [0, 1, 3], h, c, g, rtol=1e-8, max_iters=200)
    assert rb.status == B.LX_OK and rb.stats["depth"] == depth and r1.stats["depth"] == 1
    spec = [(0, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(ob, rb.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)
    if rb.iters == r1.iters:
        assert max(rel(a, b) for a, b in zip(ob, o1)) <= 1e-13
    # windows: ceil(max iters / depth), plus one re-execution per window in
    # which an output stopped
    its = rb.iters
    windows = (max(its) + depth - 1) // depth
    stops = len({(i - 1) // depth for i in its})
    assert rb.stats["n_launch"] == windows + stops
    # a re-execution recomputes up to the last term taken by an output that
    # stopped in its window
    redo = {}
    for i in its:
        wi = (i - 1) // depth
        redo[wi] = max(redo.get(wi, 0), i - wi * depth)
    assert rb.stats["n_apply"] == depth * windows + sum(redo.values())


@pytest.mark.parametrize("depth", [3, 4, 6])
@pytest.mark.parametrize("nx,ny", [(6, 5), (4, 3), (130, 7), (256, 40), (8, 6)])
def test_windows_small_and_odd_grids(ctx, depth, nx, ny):
    """Grids narrower than a tile and than the halo (indices wrap several
    times), an odd number of rows, a single partial tile row; four outputs."""
    prm, h = diffadv_setup(nx, ny, cfl=20.0)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(nx * 100 + ny).standard_normal((ny, nx))
    say("window small grid", depth, nx, ny)
    r, o = _solve(ctx, depth, 16, 0, _op(prm), v, [0, 2, 1, 3], h, c, g, rtol=1e-9, max_iters=300)
    # sides shorter than the window's halo run two iterations per launch
    assert r.status == B.LX_OK and r.stats["depth"] == (depth if min(nx, ny) >= depth else 2)
    spec = [(0, 1.0, 1.0), (2, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)


@pytest.mark.parametrize("depth", [3, 4, 6])
@pytest.mark.parametrize("max_iters", [1, 2, 3, 4, 5, 6, 7, 9, 13])
def test_windows_at_max_iters(ctx, depth, max_iters):
    """The budget ends at every position inside a window: LX_ENOTCONV with
    exactly max_iters terms."""
    prm, h = diffadv_setup(96, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(4).standard_normal((64, 96))
    say("window notconv", depth, max_iters)
    r, o = _solve(ctx, depth, 16, 0, _op(prm), v, [0, 2], h, c, g, rtol=1e-12, max_iters=max_iters,
                  raise_on_error=False)
    assert r.status == B.LX_ENOTCONV and r.iters == [max_iters, max_iters]
    ref = leja_phi(_A(prm), v, [(0, 1.0, 1.0), (2, 1.0, 1.0)], h, c, g, 1e-12, 0.0, max_iters)
    assert max(rel(a, b) for a, b in zip(o, ref.p)) <= PARITY


@pytest.mark.parametrize("depth", [3, 4, 6])
def test_windows_edge_inputs(ctx, depth):
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    say("window zero / nan", depth)
    r, o = _solve(ctx, depth, 16, 0, _op(prm), np.zeros((64, 64)), [1], h, c, g, rtol=1e-8)
    assert r.status == B.LX_OK and r.iters == [1] and not np.any(o[0])
    v = np.ones((64, 64))
    v[10, 11] = np.nan
    r, o = _solve(ctx, depth, 16, 0, _op(prm), v, [0], h, c, g, raise_on_error=False)
    assert r.status == B.LX_ENONFINITE


@pytest.mark.parametrize("depth", [3, 4, 6])
def test_windows_1024_squared_workload(ctx, depth):
    p, v = W.config2(n=1024)
    op = B.make_operator(p)
    x0 = W.start_vector(p.n)
    say("1024^2 phi123 windows", depth)
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    r, o = _solve(ctx, depth, 16, 0, op, v, [1, 2, 3], p.h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK and r.stats["depth"] == depth
    A = _A(dict(D=p.D, vx=p.vx, vy=p.vy, dx=p.dx, dy=p.dy))
    spec = [(1, 1.0, 1.0), (2, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(A, v, spec, p.h, c, g, 1e-8, 0.0, 200, f), PARITY)
    for l, ob in zip([1, 2, 3], o):
        ex = phi_fft(v, l, p.h, p.D, p.vx, p.vy, p.dx, p.dy)
        assert rel(ob, ex) <= 1e-7


@pytest.mark.parametrize("depth,th", [(3, 16), (4, 8), (4, 16), (6, 16)])
def test_burgers_jacobian_windows(ctx, depth, th):
    """The Burgers state staged beside y_m in every window; six falls back
    to four for this operator."""
    n, ny = 130, 90
    ub = W.fourier_modes(n, seed=5)[:ny, :]
    nu = 2e-3
    op_b = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=n, ny=ny, dx=1 / n, dy=1 / ny, nu=nu)
    vb = np.random.default_rng(2).standard_normal((ny, n))
    hb = 5.0 * W.burgers_cfl_step(nu, float(np.max(np.abs(ub))), 1 / n, 1 / ny)
    rho = 2.0 / W.burgers_cfl_step(nu, float(np.max(np.abs(ub))), 1 / n, 1 / ny)
    cb, gb = -1.05 * rho / 2.0, 1.05 * rho / 4.0
    say("burgers window", depth, th)
    outs = [dev(np.zeros((ny, n))) for _ in range(2)]
    ctx.set_depth(depth, th, 0)
    try:
        r = ctx.phi_leja(op_b, dev(vb), outs, [1, 2], hb, cb, gb, u=dev(ub), rtol=1e-8, max_iters=200)
    finally:
        ctx.set_depth(0)
    assert r.status == B.LX_OK and r.stats["depth"] == min(depth, 4)
    Ab = lambda w: burgers_J(ub, w, nu, 1 / n, 1 / ny)
    oracle_parity([host(o) for o in outs], r.iters,
                  lambda f: leja_phi(Ab, vb, [(1, 1.0, 1.0), (2, 1.0, 1.0)], hb, cb, gb, 1e-8, 0.0, 200, f), PARITY)


@pytest.mark.parametrize("scheme", ["exprb42", "exprb32"])
def test_integrator_steps_with_windows(ctx, scheme):
    from oracle.phi_action import exprb32_step, exprb42_step
    n = 128
    nu = 2e-3
    u0 = W.fourier_modes(n, seed=3)
    umax = float(np.max(np.abs(u0)))
    h = 2.0 * W.burgers_cfl_step(nu, umax, 1 / n, 1 / n)
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=nu)
    say("integrator windows", scheme)
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(W.start_vector(n)), iters=20)
    out = dev(np.zeros((n, n)))
    ctx.set_depth(4)
    try:
        code = {"exprb42": B.LX_EXPRB42, "exprb32": B.LX_EXPRB32}[scheme]
        r = ctx.exprb_step(op, dev(u0), out, h, c, g, rtol=1e-10, max_iters=300, scheme=code)
    finally:
        ctx.set_depth(0)
    assert r.status == B.LX_OK and r.stats["depth"] == 4
    step = {"exprb42": exprb42_step, "exprb32": exprb32_step}[scheme]
    oracle_step_parity(host(out), r.iters,
                       lambda f: step(u0, nu, 1 / n, 1 / n, h, c, g, 1e-10, 0.0, 300, force_iters=f), PARITY)


def test_windows_repeat_bitwise_and_other_operators_fall_back(ctx):
    prm, h = diffadv_setup(192, 160)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(3).standard_normal((160, 192))
    say("window determinism")
    r1, o1 = _solve(ctx, 4, 16, 0, _op(prm), v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    r2, o2 = _solve(ctx, 4, 16, 0, _op(prm), v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    assert r1.iters == r2.iters and all(np.array_equal(a, b) for a, b in zip(o1, o2))
    # the Burgers Jacobian runs windows of four when six are asked
    n = 64
    ub = W.fourier_modes(n, seed=5)
    opb = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=2e-2)
    hb = 2.0 * W.burgers_cfl_step(2e-2, float(np.max(np.abs(ub))), 1 / n, 1 / n)
    rho = 2.0 / W.burgers_cfl_step(2e-2, float(np.max(np.abs(ub))), 1 / n, 1 / n)
    out = dev(np.zeros((n, n)))
    ctx.set_depth(6)
    try:
        rb = ctx.phi_leja(opb, dev(ub), [out], [1], hb, -1.05 * rho / 2, 1.05 * rho / 4, u=dev(ub), rtol=1e-8)
    finally:
        ctx.set_depth(0)
    assert rb.status == B.LX_OK and rb.stats["depth"] == 4
    ref = leja_phi(lambda w: burgers_J(ub, w, 2e-2, 1 / n, 1 / n), ub, [(1, 1.0, 1.0)], hb, -1.05 * rho / 2,
                   1.05 * rho / 4, 1e-8, 0.0, 500)
    assert rel(host(out), ref.p[0]) <= 1e-9


@pytest.mark.parametrize("nx,ny", [(200, 136), (64, 64), (6, 5), (130, 20)])
@pytest.mark.parametrize("iters", [1, 2, 5, 8, 20])
def test_blocked_power_iteration_matches_oracle(ctx, nx, ny, iters):
    """Four power sweeps per launch (the last launch takes the rest), the
    norms deferred to the launch boundary: rho_hat as the oracle's
    normalised iteration."""
    prm, _ = diffadv_setup(nx, ny, D=0.7, vx=-30.0, vy=45.0)
    x0 = np.random.default_rng(nx + 7 * ny + iters).standard_normal((ny, nx))
    say("blocked power", nx, ny, iters)
    ctx.set_window_kernel(1)   # LDS tiles (register marching is the default where it applies)
    try:
        rho, c, g = ctx.spectrum(_op(prm), x0=dev(x0), iters=iters)
        st = ctx.stats()
    finally:
        ctx.set_window_kernel(0)
    assert st["depth"] == 4 and st["n_launch"] == (iters + 3) // 4
    rho_o, _ = power_iteration(_A(prm), x0, iters)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


@pytest.mark.parametrize("nx,ny,iters", [(128, 128, 20), (200, 136, 7), (64, 40, 5), (6, 5, 3), (130, 20, 1),
                                         (97, 64, 6)])
def test_blocked_power_iteration_burgers_jacobian(ctx, nx, ny, iters):
    """The Burgers Jacobian at a seeded state: four sweeps per launch with u
    staged beside the basis (even nx of at least four cells), one sweep per
    launch for odd nx; rho_hat as the oracle's normalised iteration."""
    rng = np.random.default_rng(nx * 31 + ny + iters)
    u = rng.standard_normal((ny, nx))
    x0 = rng.standard_normal((ny, nx))
    nu, dx, dy = 2e-2, 1.0 / nx, 1.0 / ny
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=nx, ny=ny, dx=dx, dy=dy, nu=nu)
    say("blocked power burgers", nx, ny, iters)
    rho, _, _ = ctx.spectrum(op, u=dev(u), x0=dev(x0), iters=iters)
    st = ctx.stats()
    if nx % 2 == 0:
        assert st["depth"] == 4 and st["n_launch"] == (iters + 3) // 4
    else:
        assert st["depth"] == 1 and st["n_launch"] == iters
    rho_o, _ = power_iteration(lambda w: burgers_J(u, w, nu, dx, dy), x0, iters)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


@pytest.mark.parametrize("depth", [3, 4, 6])
def test_windows_with_the_largest_budget(ctx, depth):
    """max_iters = LX_MAX_ITERS: the window past the budget reads Leja
    points and coefficients up to d_{max_iters + depth}."""
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(12).standard_normal((64, 64))
    say("window largest budget", depth)
    r, o = _solve(ctx, depth, 16, 0, _op(prm), v, [0, 3], h, c, g, rtol=1e-10, max_iters=B.LX_MAX_ITERS)
    assert r.status == B.LX_OK and r.stats["depth"] == depth
    spec = [(0, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-10, 0.0, 300, f), PARITY)
