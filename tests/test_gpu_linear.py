"""GPU parity of the third-order upwind operator and the linear-problem
step (Sec. 3, Problems I and II) against the CPU oracle, through the C ABI.

Bar as in the other parity tests: relative L2 error <= 1e-10 in FP64 with
equal iteration counts (a borderline stop decision that flips by one sweep
is rerun on the oracle at the GPU's count); the radius-2 stencil is checked
with one and two iterations per launch, on ragged tiles, on grids narrower
than a tile (indices wrap several times) and with both signs of v; the
paper-shaped problems against the oracle's step and the exact solution.
"""
import numpy as np
import pytest

from oracle.exact import diffadv3_symbol, linear_step_fft
from oracle.operators import diffadv3_apply
from oracle.phi_action import leja_phi, linear_step, power_iteration, shift_scale
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import dev, host, oracle_parity, rel, say

pytestmark = pytest.mark.gpu

PARITY = 1e-10


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=2048 * 2048, k_max=4)
    yield c
    c.close()


def _setup(nx, ny, D=1.0, vx=None, vy=None, cfl=20.0):
    dx, dy = 1.0 / nx, 1.0 / ny
    vx = 2.0 * D / dx if vx is None else vx
    vy = 2.0 * D / dy if vy is None else vy
    h = cfl * W.diffadv3_cfl_step(D, vx, vy, dx, dy)
    prm = dict(nx=nx, ny=ny, dx=dx, dy=dy, D=D, vx=vx, vy=vy)
    op = B.make_operator(kind=B.LX_OP_DIFFADV2D_UP3, nx=nx, ny=ny, dx=dx, dy=dy, D=D, vx=vx, vy=vy)
    A = lambda y: diffadv3_apply(y, D, vx, vy, dx, dy)
    return prm, op, A, h


def _shift(A, shape, seed=7):
    rho, _ = power_iteration(A, np.random.default_rng(seed).standard_normal(shape), 20)
    return shift_scale(rho)


def _solve(ctx, depth, th, nb, op, v, ls, h, c, g, **kw):
    outs = [dev(np.zeros(v.shape)) for _ in ls]
    ctx.set_depth(depth, th, nb)
    try:
        r = ctx.phi_leja(op, dev(v), outs, ls, h, c, g, **kw)
    finally:
        ctx.set_depth(0)
    return r, [host(o) for o in outs]


@pytest.mark.parametrize("nx,ny,vx,vy", [(64, 64, None, None), (97, 75, -30.0, 50.0), (200, 136, 40.0, -70.0),
                                         (4, 5, 3.0, -2.0)])
def test_up3_spectrum_matches_oracle(ctx, nx, ny, vx, vy):
    prm, op, A, _ = _setup(nx, ny, vx=vx, vy=vy)
    x0 = np.random.default_rng(nx + ny).standard_normal((ny, nx))
    say("spectrum up3", nx, ny, vx, vy)
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    rho_o, _ = power_iteration(A, x0, 20)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


# (depth, th, nb): one iteration per launch; two on 8- and 16-row tiles,
# one workgroup per tile and fewer workgroups than tiles
SHAPES = [(1, 0, 0), (2, 8, 0), (2, 16, 0), (2, 16, 8), (2, 8, 24), (3, 8, 0), (3, 16, 8), (4, 8, 0), (4, 16, 0)]


@pytest.mark.parametrize("depth,th,nb", SHAPES)
@pytest.mark.parametrize("vx,vy", [(None, None), (-90.0, 60.0), (35.0, -120.0)])
def test_up3_phi_matches_oracle(ctx, depth, th, nb, vx, vy):
    """Ragged tiles both ways (200 = 128 + 72 columns, 136 rows), phi_0,
    phi_1 and phi_3 from one basis, each sign of v on each axis."""
    prm, op, A, h = _setup(200, 136, vx=vx, vy=vy)
    c, g = _shift(A, (136, 200))
    v = np.random.default_rng(11).standard_normal((136, 200))
    say("up3 phi", depth, th, nb, vx, vy)
    r, o = _solve(ctx, depth, th, nb, op, v, [0, 1, 3], h, c, g, rtol=1e-9, max_iters=300)
    assert r.status == B.LX_OK and r.stats["depth"] == depth   # depth 4 runs 8-row tiles when 16 are asked
    spec = [(0, 1.0, 1.0), (1, 1.0, 1.0), (3, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(A, v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)


@pytest.mark.parametrize("nx,ny", [(4, 4), (6, 5), (130, 7), (97, 75), (256, 40), (8, 8), (12, 9)])
@pytest.mark.parametrize("depth", [4, 3, 2, 1])
def test_up3_small_and_odd_grids(ctx, nx, ny, depth):
    """Grids narrower than a tile and than the 4-cell halo reach, odd sides
    (odd nx runs one iteration per launch whatever is asked)."""
    prm, op, A, h = _setup(nx, ny, vx=-2.0 * nx, vy=1.5 * ny, cfl=10.0)
    c, g = _shift(A, (ny, nx))
    v = np.random.default_rng(nx * 100 + ny).standard_normal((ny, nx))
    say("up3 small grid", nx, ny, depth)
    r, o = _solve(ctx, depth, 16, 0, op, v, [0, 2], h, c, g, rtol=1e-9, max_iters=300)
    assert r.status == B.LX_OK
    # odd nx: one iteration per launch; windows need sides of 2 depth cells
    want = 1 if nx % 2 else (depth if depth <= 2 or min(nx, ny) >= 2 * depth else 2)
    assert r.stats["depth"] == want
    spec = [(0, 1.0, 1.0), (2, 1.0, 1.0)]
    oracle_parity(o, r.iters, lambda f: leja_phi(A, v, spec, h, c, g, 1e-9, 0.0, 300, f), PARITY)


def test_up3_depths_agree_and_tile_rows_capped(ctx):
    """Two iterations per launch give the one-iteration results (same
    iteration counts: same terms in the same order, up to the order of the
    norm reductions); asking for 32-row tiles runs 16-row ones."""
    prm, op, A, h = _setup(256, 192, vx=50.0, vy=-80.0, cfl=50.0)
    c, g = _shift(A, (192, 256))
    v = np.random.default_rng(5).standard_normal((192, 256))
    say("up3 depth compare")
    r2, o2 = _solve(ctx, 2, 32, 0, op, v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=300)
    r1, o1 = _solve(ctx, 1, 0, 0, op, v, [1, 2, 3], h, c, g, rtol=1e-8, max_iters=300)
    assert r2.stats["depth"] == 2 and r1.stats["depth"] == 1
    if r2.iters == r1.iters:
        assert max(rel(a, b) for a, b in zip(o2, o1)) <= 1e-13


@pytest.mark.parametrize("iters", [1, 6, 20])
def test_up3_blocked_power_iteration(ctx, iters):
    prm, op, A, _ = _setup(136, 72, vx=-40.0, vy=90.0)
    x0 = np.random.default_rng(iters).standard_normal((72, 136))
    say("up3 blocked power", iters)
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=iters)
    assert ctx.stats()["depth"] == 4
    rho_o, _ = power_iteration(A, x0, iters)
    assert abs(rho - rho_o) <= 1e-12 * rho_o


def test_up3_fp32_sweeps_within_tolerance(ctx):
    prm, op, A, h = _setup(160, 96, vx=40.0, vy=25.0, cfl=20.0)
    op32 = B.make_operator(kind=B.LX_OP_DIFFADV2D_UP3, nx=160, ny=96, dx=prm["dx"], dy=prm["dy"], D=1.0,
                           vx=40.0, vy=25.0, prec=B.LX_FP32_SWEEP)
    c, g = _shift(A, (96, 160))
    v = np.random.default_rng(8).standard_normal((96, 160))
    out = dev(np.zeros((96, 160)))
    say("up3 fp32")
    r = ctx.phi_leja(op32, dev(v), [out], [1], h, c, g, rtol=1e-6, max_iters=300)
    assert r.status == B.LX_OK and r.stats["n_fp32"] > 0
    ref = leja_phi(A, v, [(1, 1.0, 1.0)], h, c, g, 1e-12, 0.0, 300)
    assert rel(host(out), ref.p[0]) <= 1e-5


@pytest.mark.parametrize("source", [False, True])
@pytest.mark.parametrize("n,cfl,depth", [(128, 10.0, 2), (128, 100.0, 2), (250, 10.0, 2), (250, 10.0, 1), (75, 1.0, 2),
                                         (128, 100.0, 4), (250, 10.0, 3)])
def test_linear_step_matches_oracle(ctx, n, cfl, depth, source):
    """Problems I and II on [-1, 1)^2 (nu = 10, the paper's initial data and
    source), tolerance 1e-12: the step against the oracle's step, with the
    shift from the library's own power iteration."""
    p, u0, S = W.paper_linear(n, cfl, source)
    op = B.make_operator(p)
    A = lambda y: diffadv3_apply(y, p.D, p.vx, p.vy, p.dx, p.dy)
    x0 = W.start_vector(n)
    say("linear step", n, cfl, depth, source)
    rho, c, g = ctx.spectrum(op, x0=dev(x0), iters=20)
    out = dev(np.zeros((n, n)))
    ctx.set_depth(depth)
    try:
        r = ctx.linear_step(op, dev(u0), out, p.h, c, g, source=None if S is None else dev(S), rtol=1e-12,
                            max_iters=400)
    finally:
        ctx.set_depth(0)
    assert r.status == B.LX_OK
    assert r.stats["depth"] == (depth if n % 2 == 0 else 1)

    def run(force):
        # the oracle's linear step, with the phi pass forced to the GPU's
        # count when a borderline stop decision flipped
        w = u0 if S is None else p.h * (A(u0) + S)
        lr = leja_phi(A, w, [(0 if S is None else 1, 1.0, 1.0)], p.h, c, g, 1e-12, 0.0, 400, force)
        if force is None:
            ref = linear_step(A, u0, S, p.h, c, g, 1e-12, 0.0, 400)
            assert np.array_equal(ref.u_next, u0 + lr.p[0] if S is not None else lr.p[0])
        lr.p = [lr.p[0] if S is None else u0 + lr.p[0]]
        return lr

    oracle_parity([host(out)], r.iters, run, PARITY)
    lam = diffadv3_symbol(n, n, p.D, p.vx, p.vy, p.dx, p.dy)
    assert rel(host(out), linear_step_fft(u0, S, p.h, lam)) <= 1e-10


def test_linear_step_2048_against_exact_solution(ctx):
    """A full time loop of Problem II at 2048^2 (h = 10 x CFL, five steps):
    every step against the exact solution, mode by mode, of the same step."""
    n = 2048
    p, u0, S = W.paper_linear(n, 10.0, True)
    op = B.make_operator(p)
    lam = diffadv3_symbol(n, n, p.D, p.vx, p.vy, p.dx, p.dy)
    say("linear step 2048 loop")
    rho, c, g = ctx.spectrum(op, x0=dev(W.start_vector(n)), iters=20)
    u, out, Sd = dev(u0), dev(np.zeros((n, n))), dev(S)
    exact = u0
    for k in range(5):
        r = ctx.linear_step(op, u, out, p.h, c, g, source=Sd, rtol=1e-12, max_iters=400)
        assert r.status == B.LX_OK
        exact = linear_step_fft(exact, S, p.h, lam)
        e = rel(host(out), exact)
        say("step", k, "iters", r.iters, "rel err vs exact", e)
        assert e <= 1e-10
        u, out = out, u
    # mean: A conserves the sum, so each step adds h * mean(S) exactly
    assert abs(float(np.mean(host(u))) - (float(np.mean(u0)) + 5 * p.h * float(np.mean(S)))) <= 1e-12


def test_linear_step_rejects_other_operators(ctx):
    n = 64
    u = dev(np.ones((n, n)))
    out = dev(np.zeros((n, n)))
    opb = B.make_operator(kind=B.LX_OP_BURGERS2D, n=n, nu=1e-3)
    say("linear step invalid")
    r = ctx.linear_step(opb, u, out, 1e-3, -1.0, 0.5, raise_on_error=False)
    assert r.status == B.LX_EINVAL
    op3 = B.make_operator(kind=B.LX_OP_DIFFADV2D_UP3, nx=3, ny=8, D=1.0)
    r = ctx.linear_step(op3, dev(np.ones((8, 3))), dev(np.zeros((8, 3))), 1e-3, -1.0, 0.5, raise_on_error=False)
    assert r.status == B.LX_EINVAL
    r = ctx.linear_step(B.make_operator(kind=B.LX_OP_DIFFADV2D_UP3, n=n, D=1.0), u, u, 1e-3, -1.0, 0.5,
                        raise_on_error=False)
    assert r.status == B.LX_EINVAL
