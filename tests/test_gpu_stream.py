"""GPU parity of the register-marching kernels (`leja_stream` windows of
four, six and eight Leja iterations per launch, `power_stream` power
iteration) against the CPU oracle, the exact Fourier solution and the
LDS-tile window kernel, through the C ABI.

Each output must take exactly the terms of the one-iteration loop: the
oracle comparison at 1e-10 (a borderline stop decision flipped by the order
of the norm reductions is rerun at the GPU's count and reported), bitwise
equality with the LDS-tile windows when the counts agree (both form every
level with the same operand order), stops at every position inside a window,
forced band and workgroup counts (items per wavefront > 1, idle wavefronts),
ragged and tiny grids.
"""
import numpy as np
import pytest

from oracle.exact import phi_fft
from oracle.operators import diffadv_apply
from oracle.phi_action import leja_phi, power_iteration
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import closed_form_shift, dev, diffadv_setup, host, oracle_parity, rel, say

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


def _solve(ctx, depth, kind, bands, nb, op, v, ls, h, c, g, **kw):
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, 0, 0)
    ctx.set_window_kernel(kind, bands, nb)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, **kw)
    finally:
        ctx.set_depth(0)
        ctx.set_window_kernel(0)
    return r, [host(o) for o in outs]


CASES = [(4, [0, 1, 3, 2]), (6, [0, 1, 3]), (6, [2]), (8, [1]), (8, [0, 1, 3]), (8, [2, 3]), (4, [1])]


@pytest.mark.parametrize("depth,ls", CASES)
@pytest.mark.parametrize("bands,nb", [(0, 0), (3, 0), (7, 2), (136, 1)])
def test_stream_windows_match_oracle_and_tiles(ctx, depth, ls, bands, nb):
    """Ragged strips both ways (200 columns, 136 rows); outputs stop in
    different windows; several items per wavefront when bands and
    workgroups are forced."""
    prm, h = diffadv_setup(200, 136)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(31).standard_normal((136, 200))
    say("stream window", depth, ls, bands, nb)
    rs, os_ = _solve(ctx, depth, 2, bands, nb, _op(prm), v, ls, h, c, g, rtol=1e-8, max_iters=200)
    assert rs.status == B.LX_OK and rs.stats["depth"] == depth
    spec = [(l, 1.0, 1.0) for l in ls]
    oracle_parity(os_, rs.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)
    its = rs.iters
    windows = (max(its) + depth - 1) // depth
    stops = len({(i - 1) // depth for i in its})
    assert rs.stats["n_launch"] == windows + stops
    if depth <= 6 and len(ls) <= (3 if depth == 6 else 4):
        # the LDS-tile windows of the same depth take the same terms in the
        # same order with the same stencil bits
        rt, ot = _solve(ctx, depth, 1, 0, 0, _op(prm), v, ls, h, c, g, rtol=1e-8, max_iters=200)
        if rt.iters == rs.iters:
            assert all(np.array_equal(a, b) for a, b in zip(os_, ot))


@pytest.mark.parametrize("ls", [[0, 1, 3], [1, 2, 3], [2, 3]])
def test_stream_depth8_matches_depth4_bitwise(ctx, ls):
    """Every depth takes each output's terms in the same order with the
    same operations, so windows of eight (the first-window kernel, the
    one-output forms of the last windows and re-executions) and of four
    give the same bits whenever the iteration counts agree; outputs stop in
    different windows here."""
    prm, h = diffadv_setup(200, 136)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(77).standard_normal((136, 200))
    say("stream depth 8 vs 4", ls)
    r8, o8 = _solve(ctx, 8, 2, 0, 0, _op(prm), v, ls, h, c, g, rtol=1e-8, max_iters=200)
    r4, o4 = _solve(ctx, 4, 2, 0, 0, _op(prm), v, ls, h, c, g, rtol=1e-8, max_iters=200)
    assert r8.status == B.LX_OK and r8.stats["depth"] == 8 and r4.stats["depth"] == 4
    spec = [(l, 1.0, 1.0) for l in ls]
    oracle_parity(o8, r8.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-8, 0.0, 200, f), PARITY)
    if r8.iters == r4.iters:
        assert all(np.array_equal(a, b) for a, b in zip(o8, o4))


@pytest.mark.parametrize("depth", [4, 6, 8])
@pytest.mark.parametrize("nx,ny", [(8, 8), (10, 12), (64, 9), (130, 20), (256, 40), (14, 200)])
def test_stream_small_and_odd_grids(ctx, depth, nx, ny):
    """Strips wider than the grid (columns wrap several times), an odd
    number of rows, a single band; sides shorter than the window fall back."""
    prm, h = diffadv_setup(nx, ny, cfl=20.0)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(nx * 100 + ny).standard_normal((ny, nx))
    ls = {4: [0, 2], 6: [0, 1, 3], 8: [0, 1, 3]}[depth]
    say("stream small grid", depth, nx, ny)
    r, o = _solve(ctx, depth, 2, 0, 0, _op(prm), v, ls, h, c, g, rtol=1e-9, max_iters=300)
    assert r.status == B.LX_OK
    if min(nx, ny) >= depth:
        assert r.stats["depth"] == depth
    spec = [(l, 1.0, 1.0) for l in ls]
    oracle_parity(o, r.iters, lambda f: leja_phi(_A(prm), v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)


@pytest.mark.parametrize("depth,K", [(4, 2), (6, 2), (6, 3), (8, 1), (8, 2), (8, 3)])
@pytest.mark.parametrize("max_iters", [1, 2, 3, 4, 5, 6, 7, 8, 9, 13])
def test_stream_windows_at_max_iters(ctx, depth, K, max_iters):
    """The budget ends at every position inside a window: LX_ENOTCONV with
    exactly max_iters terms (the re-execution takes fewer than D terms)."""
    prm, h = diffadv_setup(96, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(4).standard_normal((64, 96))
    ls = [0, 2, 3][:K] if K > 1 else [2]
    say("stream notconv", depth, max_iters)
    r, o = _solve(ctx, depth, 2, 0, 0, _op(prm), v, ls, h, c, g, rtol=1e-12, max_iters=max_iters,
                  raise_on_error=False)
    assert r.status == B.LX_ENOTCONV and r.iters == [max_iters] * len(ls)
    ref = leja_phi(_A(prm), v, [(l, 1.0, 1.0) for l in ls], h, c, g, 1e-12, 0.0, max_iters)
    assert max(rel(a, b) for a, b in zip(o, ref.p)) <= PARITY


@pytest.mark.parametrize("depth", [4, 6, 8])
def test_stream_edge_inputs(ctx, depth):
    prm, h = diffadv_setup(64, 64)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    say("stream zero / nan", depth)
    r, o = _solve(ctx, depth, 2, 0, 0, _op(prm), np.zeros((64, 64)), [1], h, c, g, rtol=1e-8)
    assert r.status == B.LX_OK and r.iters == [1] and not np.any(o[0])
    v = np.ones((64, 64))
    v[10, 11] = np.nan
    r, o = _solve(ctx, depth, 2, 0, 0, _op(prm), v, [0], h, c, g, raise_on_error=False)
    assert r.status == B.LX_ENONFINITE


@pytest.mark.parametrize("depth,ls", [(6, [1, 2, 3]), (4, [1, 2, 3]), (8, [1]), (8, [1, 2, 3])])
def test_stream_1024_squared_workload(ctx, depth, ls):
    """The 1024^2 phi_1..phi_3 workload: oracle parity and the exact Fourier
    solution within 10 x tol."""
    p, v = W.config2(n=1024)
    op = B.make_operator(p)
    x0 = W.start_vector(p.n)
    say("1024^2 stream windows", depth, ls)
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    r, o = _solve(ctx, depth, 2, 0, 0, op, v, ls, p.h, c, g, rtol=1e-8, max_iters=200)
    assert r.status == B.LX_OK and r.stats["depth"] == depth
    A = _A(dict(D=p.D, vx=p.vx, vy=p.vy, dx=p.dx, dy=p.dy))
    spec = [(l, 1.0, 1.0) for l in ls]
    oracle_parity(o, r.iters, lambda f: leja_phi(A, v, spec, p.h, c, g, 1e-8, 0.0, 200, f), PARITY)
    for l, ob in zip(ls, o):
        ex = phi_fft(v, l, p.h, p.D, p.vx, p.vy, p.dx, p.dy)
        assert rel(ob, ex) <= 1e-7


def test_stream_repeat_bitwise(ctx):
    prm, h = diffadv_setup(192, 160)
    c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
    v = np.random.default_rng(3).standard_normal((160, 192))
    say("stream determinism")
    r1, o1 = _solve(ctx, 6, 2, 0, 0, _op(prm), v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    r2, o2 = _solve(ctx, 6, 2, 0, 0, _op(prm), v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=200)
    assert r1.iters == r2.iters and all(np.array_equal(a, b) for a, b in zip(o1, o2))


@pytest.mark.parametrize("nx,ny", [(200, 136), (64, 64), (10, 10), (130, 20), (1024, 1024)])
@pytest.mark.parametrize("iters", [1, 2, 5, 10, 11, 20, 23])
def test_stream_power_iteration_matches_oracle(ctx, nx, ny, iters):
    """Up to ten power sweeps per launch by register marching (the last
    launch takes the rest), the norms deferred to the launch boundary:
    rho_hat as the oracle's normalised iteration."""
    prm, _ = diffadv_setup(nx, ny, D=0.7, vx=-30.0, vy=45.0)
    x0 = np.random.default_rng(nx + 7 * ny + iters).standard_normal((ny, nx))
    say("stream power", nx, ny, iters)
    ctx.set_window_kernel(2)
    try:
        rho, c, g = ctx.spectrum(_op(prm), x0=dev(x0), iters=iters)
        st = ctx.stats()
    finally:
        ctx.set_window_kernel(0)
    per = st["depth"]
    assert 1 <= per <= 10 and st["n_launch"] == (iters + per - 1) // per
    rho_o, _ = power_iteration(_A(prm), x0, iters)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


@pytest.mark.parametrize("scale", [1e-110, 1e-90, 1.0, 1e5, 1e15])
def test_stream_power_iteration_start_vector_scale(ctx, scale):
    """The first launch takes the start vector unscaled and measures its
    norm itself when ||x0||^2 lies in [1e-200, 1e20]; outside that range
    (here 1e-110 and 1e15 on 200 x 136 N(0,1) values) the iteration runs
    again with x0 scaled first.  Either way rho_hat is the normalised
    iteration's, which does not depend on the scale of x0."""
    nx, ny, iters = 200, 136, 20
    prm, _ = diffadv_setup(nx, ny, D=0.7, vx=-30.0, vy=45.0)
    x0 = np.random.default_rng(17).standard_normal((ny, nx))
    say("stream power, start vector scaled by", scale)
    ctx.set_window_kernel(2)
    try:
        rho, _, _ = ctx.spectrum(_op(prm), x0=dev(scale * x0), iters=iters)
    finally:
        ctx.set_window_kernel(0)
    rho_o, _ = power_iteration(_A(prm), x0, iters)
    assert np.isfinite(rho) and abs(rho - rho_o) <= 1e-12 * rho_o


# ---------------------------------------------------------------------------
# the Burgers Jacobian, and FP32 sweeps, by register marching
# ---------------------------------------------------------------------------

def _burgers_case(nx, ny, seed, pe=2.0, cfl=5.0):
    from oracle.operators import burgers_J
    u = W.fourier_modes(max(nx, ny), seed=seed)[:ny, :nx] + 0.2
    umax = float(np.max(np.abs(u)))
    dx, dy = 1.0 / nx, 1.0 / ny
    nu = umax * max(dx, dy) / pe
    h = cfl * W.burgers_cfl_step(nu, umax, dx, dy)
    rho = 2.0 / W.burgers_cfl_step(nu, umax, dx, dy)
    c, g = -1.05 * rho / 2.0, 1.05 * rho / 4.0
    op = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=nx, ny=ny, dx=dx, dy=dy, nu=nu)
    A = lambda w: burgers_J(u, w, nu, dx, dy)
    v = np.random.default_rng(seed + 100).standard_normal((ny, nx))
    return op, A, u, v, h, c, g


def _solve_u(ctx, depth, kind, op, u, v, ls, h, c, g, **kw):
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, 0, 0)
    ctx.set_window_kernel(kind)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, u=dev(u), **kw)
    finally:
        ctx.set_depth(0)
        ctx.set_window_kernel(0)
    return r, [host(o) for o in outs]


@pytest.mark.parametrize("depth,ls", [(4, [1]), (4, [0, 3]), (6, [2])])
@pytest.mark.parametrize("nx,ny", [(200, 136), (128, 128), (10, 12), (66, 34)])
def test_stream_burgers_windows_match_oracle_and_tiles(ctx, depth, ls, nx, ny):
    """The Burgers Jacobian by register marching (the state u staged row by
    row beside level 0): the oracle at 1e-10, and bitwise the LDS-tile
    windows of four (the same stencil operands in the same order) when the
    iteration counts agree."""
    op, A, u, v, h, c, g = _burgers_case(nx, ny, nx + ny)
    say("stream burgers", depth, ls, nx, ny)
    r, o = _solve_u(ctx, depth, 2, op, u, v, ls, h, c, g, rtol=1e-9, max_iters=300)
    assert r.status == B.LX_OK and r.stats["depth"] == depth and r.stats["marching"] == 1
    spec = [(l, 1.0, 1.0) for l in ls]
    oracle_parity(o, r.iters, lambda f: leja_phi(A, v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)
    if depth == 4:
        rt, ot = _solve_u(ctx, 4, 1, op, u, v, ls, h, c, g, rtol=1e-9, max_iters=300)
        assert rt.stats["marching"] == 0
        if rt.iters == r.iters:
            assert all(np.array_equal(a, b) for a, b in zip(o, ot))


@pytest.mark.parametrize("max_iters", [1, 3, 4, 5, 8, 9])
def test_stream_burgers_windows_at_max_iters(ctx, max_iters):
    op, A, u, v, h, c, g = _burgers_case(96, 64, 5)
    say("stream burgers notconv", max_iters)
    r, o = _solve_u(ctx, 4, 2, op, u, v, [1, 2], h, c, g, rtol=1e-13, max_iters=max_iters, raise_on_error=False)
    assert r.status == B.LX_ENOTCONV and r.iters == [max_iters] * 2
    ref = leja_phi(A, v, [(1, 1.0, 1.0), (2, 1.0, 1.0)], h, c, g, 1e-13, 0.0, max_iters)
    assert max(rel(a, b) for a, b in zip(o, ref.p)) <= PARITY


@pytest.mark.parametrize("kind", ["diffadv", "burgers"])
@pytest.mark.parametrize("depth,ls", [(4, [1, 2]), (4, [0]), (6, [3])])
@pytest.mark.parametrize("switch", [1e4, 0.0])
def test_stream_fp32_windows_against_fp64_oracle(ctx, kind, depth, ls, switch):
    """FP32 sweeps in windows: the basis vectors and stencil arithmetic in
    FP32 once every term is small (fp32_switch times the tolerance; 0: from
    the first window), the outputs, terms, norms and coefficients in FP64.
    Error against the FP64 oracle within the tolerance with the default
    switch (reported for a switch of 0)."""
    if kind == "diffadv":
        prm, h = diffadv_setup(256, 192)
        c, g = closed_form_shift(prm["D"], prm["vx"], prm["vy"], prm["dx"], prm["dy"])
        op = _op(prm)
        op.prec = B.LX_FP32_SWEEP
        A, u = _A(prm), None
        v = np.random.default_rng(21).standard_normal((192, 256))
    else:
        op, A, u, v, h, c, g = _burgers_case(256, 192, 9)
        op.prec = B.LX_FP32_SWEEP
    say("stream fp32", kind, depth, ls, switch)
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, 0, 0)
    ctx.set_window_kernel(2)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, u=dev(u) if u is not None else None, rtol=1e-8,
                         max_iters=300, fp32_switch=switch)
    finally:
        ctx.set_depth(0)
        ctx.set_window_kernel(0)
    assert r.status == B.LX_OK and r.stats["marching"] == 1 and r.stats["depth"] == depth
    assert r.stats["n_fp32"] > 0 and r.stats["n_fp32"] % depth == 0
    ref = leja_phi(A, v, [(l, 1.0, 1.0) for l in ls], h, c, g, 1e-8, 0.0, 300)
    errs = [rel(host(o), q) for o, q in zip(outs, ref.p)]
    say("fp32 window errors vs fp64 oracle", errs, "iterations", r.iters, "oracle", ref.iters, "fp32 levels",
        r.stats["n_fp32"])
    assert max(errs) <= (1e-8 if switch > 0 else 1e-5)


def test_stream_fp32_exprb42_step_against_fp64_oracle(ctx):
    """One EXPRB42 step of a Burgers problem with FP32 sweeps in register-
    marching windows (both passes) against the FP64 oracle's step."""
    from oracle.phi_action import exprb42_step
    n = 192
    p, u0 = W.config3(n=n)
    op = B.make_operator(p)
    op32 = B.make_operator(p)
    op32.prec = B.LX_FP32_SWEEP
    rho, c, g = ctx.spectrum(op, u=dev(u0), x0=dev(W.start_vector(n)), iters=20)
    out = dev(np.zeros_like(u0))
    say("stream fp32 exprb42", n)
    ctx.set_depth(4)
    ctx.set_window_kernel(2)
    try:
        r = ctx.exprb_step(op32, dev(u0), out, p.h, c, g, rtol=1e-8, max_iters=200)
    finally:
        ctx.set_depth(0)
        ctx.set_window_kernel(0)
    assert r.status == B.LX_OK and r.stats["marching"] == 1 and r.stats["n_fp32"] > 0
    ref = exprb42_step(u0, p.nu, p.dx, p.dy, p.h, c, g, 1e-8, 0.0, 200)
    err = rel(host(out) - u0, ref.u_next - u0)
    say("fp32 exprb42 update error", err)
    assert err <= 1e-7
