"""GPU parity of batched phi actions (lx_phi_leja_batched) against the
oracle, instance by instance, through the C ABI.

Each instance of a batch must match a separate oracle run on its own data
(relative L2 <= 1e-10, equal sweep counts up to a borderline stop
decision).  Batches mix grid sizes (including odd and ragged ones),
operators, phi orders and steps; the full 256-instance workload is checked
on a sample against the oracle and on every instance through the sum
invariant.
"""
import math

import numpy as np
import pytest

from oracle.operators import burgers_J, diffadv_apply
from oracle.phi_action import leja_phi, power_iteration, shift_scale
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import dev, host, oracle_parity, rel, say

pytestmark = pytest.mark.gpu

PARITY = 1e-10


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=1 << 16, k_max=4)
    yield c
    c.close()


def splitmix_vector(seed, n):
    """splitmix64 (Steele, Lea and Flood 2014) at positions 0..n-1 of a
    stream with the given seed, mapped to [-1, 1) as the library does."""
    t = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (t + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0**-52 - 1.0


MIXED = [(64, 64, "da"), (96, 40, "da"), (33, 17, "da"), (128, 128, "bu"), (130, 66, "da"),
         (8, 8, "da"), (200, 136, "bu"), (75, 97, "da"), (256, 256, "da"), (50, 50, "bu")]
# every side even: the batch runs two iterations per launch
EVEN = [(64, 64, "da"), (96, 40, "da"), (130, 66, "da"), (128, 128, "bu"), (8, 8, "da"), (200, 136, "bu"),
        (256, 256, "da"), (50, 50, "bu"), (6, 10, "da"), (258, 34, "bu")]


def _mixed_batch(seed=0, specs=MIXED):
    rng = np.random.default_rng(seed)
    inst = []
    for i, (nx, ny, kind) in enumerate(specs):
        dx, dy = 1.0 / nx, 1.0 / ny
        v = rng.standard_normal((ny, nx))
        if kind == "da":
            D = float(np.exp(rng.uniform(np.log(0.1), np.log(10.0))))
            sp, ang = rng.uniform(0, 5), rng.uniform(0, 2 * np.pi)
            vx, vy = sp * np.cos(ang), sp * np.sin(ang)
            op = B.make_operator(kind=B.LX_OP_DIFFADV2D, nx=nx, ny=ny, dx=dx, dy=dy, D=D, vx=vx, vy=vy)
            rho = 2.0 / W.diffadv_cfl_step(D, vx, vy, dx, dy)
            A = (lambda D, vx, vy, dx, dy: (lambda y: diffadv_apply(y, D, vx, vy, dx, dy)))(D, vx, vy, dx, dy)
            u = None
        else:
            # cell Peclet number 2: the diffusion-dominated regime where the
            # real-interval Leja interpolation is stable (advection-dominated
            # Jacobians amplify rounding along the Newton basis)
            u = W.fourier_modes(max(nx, ny), seed=10 + i)[:ny, :nx] + 0.2
            nu = float(np.max(np.abs(u))) * max(dx, dy) / 2.0
            op = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=nx, ny=ny, dx=dx, dy=dy, nu=nu)
            rho = 2.0 / W.burgers_cfl_step(nu, float(np.max(np.abs(u))), dx, dy)
            A = (lambda u, nu, dx, dy: (lambda w: burgers_J(u, w, nu, dx, dy)))(u, nu, dx, dy)
        # Burgers steps stay at most 10 x CFL
        s = float(np.exp(rng.uniform(0.0, np.log(40.0 if kind == "da" else 10.0))))
        h = 2.0 * s / rho
        c, g = shift_scale(rho)
        inst.append(dict(nx=nx, ny=ny, op=op, A=A, u=u, v=v, l=int(rng.integers(0, 4)), h=h, c=c, gamma=g))
    return inst


def _run(ctx, inst, power_iters=0, x0s=None, budgets=None, **kw):
    outs = [dev(np.zeros((q["ny"], q["nx"]))) for q in inst]
    args = []
    for i, q in enumerate(inst):
        a = dict(op=q["op"], v=dev(q["v"]), out=outs[i], l=q["l"], h=q["h"], c=q["c"], gamma=q["gamma"])
        if q["u"] is not None:
            a["u"] = dev(q["u"])
        if x0s is not None and x0s[i] is not None:
            a["x0"] = dev(x0s[i])
        if budgets is not None:
            a["budget"] = budgets[i]
        args.append(a)
    st, res = ctx.phi_leja_batched(args, power_iters=power_iters, **kw)
    return st, res, [host(o) for o in outs]


def test_mixed_batch_matches_oracle_per_instance(ctx):
    inst = _mixed_batch(0)
    say("mixed batch", len(inst))
    st, res, outs = _run(ctx, inst, rtol=1e-8, max_iters=200)
    assert st == B.LX_OK
    for q, r, o in zip(inst, res, outs):
        assert r["status"] == B.LX_OK
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"],
                                              1e-8, 0.0, 200, f), PARITY)


def test_batched_power_iteration_matches_oracle(ctx):
    inst = _mixed_batch(1)
    rng = np.random.default_rng(5)
    x0s = [rng.standard_normal((q["ny"], q["nx"])) if i % 2 == 0 else None for i, q in enumerate(inst)]
    say("batched power iteration")
    st, res, outs = _run(ctx, inst, power_iters=20, x0s=x0s, rtol=1e-8, max_iters=250)
    assert st == B.LX_OK
    for i, (q, r, o) in enumerate(zip(inst, res, outs)):
        x0 = x0s[i] if x0s[i] is not None else splitmix_vector(i, q["nx"] * q["ny"]).reshape(q["ny"], q["nx"])
        rho_o, _ = power_iteration(q["A"], x0, 20)
        assert abs(r["rho_hat"] - rho_o) <= 1e-12 * rho_o, (i, r["rho_hat"], rho_o)
        c, g = shift_scale(r["rho_hat"])
        assert r["c"] == c and r["gamma"] == g
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q, c=c, g=g: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], c, g,
                                                        1e-8, 0.0, 250, f), PARITY)


def test_budgets_stop_instances_with_notconv(ctx):
    inst = _mixed_batch(2)[:5]
    budgets = [3, 0, 2, 0, 1]
    say("budgets")
    st, res, outs = _run(ctx, inst, budgets=budgets, rtol=1e-10, max_iters=200)
    assert st == B.LX_ENOTCONV
    for q, b, r, o in zip(inst, budgets, res, outs):
        if b == 0:
            assert r["status"] == B.LX_OK
            continue
        assert r["status"] == B.LX_ENOTCONV and r["iters"] == b
        ref = leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"], 1e-10, 0.0, b)
        assert rel(o, ref.p[0]) <= PARITY


def test_batch_equals_single_instance_path(ctx):
    inst = _mixed_batch(3)[:4]
    st, res, outs = _run(ctx, inst, rtol=1e-9, max_iters=200)
    for q, r, o in zip(inst, res, outs):
        out = dev(np.zeros((q["ny"], q["nx"])))
        kw = {"u": dev(q["u"])} if q["u"] is not None else {}
        rs = ctx.phi_leja(q["op"], dev(q["v"]), [out], [q["l"]], q["h"], q["c"], q["gamma"], rtol=1e-9,
                          max_iters=200, **kw)
        assert rs.iters[0] == r["iters"]
        assert rel(o, host(out)) <= 1e-12


@pytest.mark.parametrize("depth,th", [(2, 8), (2, 16), (0, 8), (0, 16)])
def test_two_iteration_batch_matches_oracle(ctx, depth, th):
    """Even sides (ragged against the 128-column tiles), both operators in
    one launch, against the oracle instance by instance; two iterations per
    launch, and the default windows of four (8-row tiles with Burgers)."""
    inst = _mixed_batch(5, EVEN)
    say("multi-iteration batch", depth, th)
    ctx.set_depth(depth, th, 0)
    try:
        st, res, outs = _run(ctx, inst, rtol=1e-8, max_iters=200)
        assert ctx.stats()["depth"] == (depth or 4)
    finally:
        ctx.set_depth(0)
    assert st == B.LX_OK
    for q, r, o in zip(inst, res, outs):
        assert r["status"] == B.LX_OK
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"],
                                              1e-8, 0.0, 200, f), PARITY)


@pytest.mark.parametrize("depth", [2, 0])
def test_two_iteration_batch_budgets_and_power_iteration(ctx, depth):
    """Budgets end at every position of a launch (two iterations) or window
    (four, the default); the batched power iteration feeds the loop."""
    ctx.set_depth(depth)
    try:
        _budgets_and_power(ctx, depth or 4)
    finally:
        ctx.set_depth(0)


def _budgets_and_power(ctx, depth):
    inst = _mixed_batch(6, EVEN)[:6]
    budgets = [3, 0, 2, 0, 1, 4] if depth == 2 else [3, 5, 2, 7, 1, 4]
    say("multi-iteration budgets", depth)
    st, res, outs = _run(ctx, inst, budgets=budgets, rtol=1e-10, max_iters=200)
    assert ctx.stats()["depth"] == depth and st == B.LX_ENOTCONV
    for q, b, r, o in zip(inst, budgets, res, outs):
        if b == 0:
            assert r["status"] == B.LX_OK
            continue
        assert r["status"] == B.LX_ENOTCONV and r["iters"] == b
        ref = leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"], 1e-10, 0.0, b)
        assert rel(o, ref.p[0]) <= PARITY
    inst = _mixed_batch(7, EVEN)
    st, res, outs = _run(ctx, inst, power_iters=20, rtol=1e-8, max_iters=250)
    assert ctx.stats()["depth"] == depth and st == B.LX_OK
    for i, (q, r, o) in enumerate(zip(inst, res, outs)):
        x0 = splitmix_vector(i, q["nx"] * q["ny"]).reshape(q["ny"], q["nx"])
        rho_o, _ = power_iteration(q["A"], x0, 20)
        assert abs(r["rho_hat"] - rho_o) <= 1e-12 * rho_o
        c, g = shift_scale(r["rho_hat"])
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q, c=c, g=g: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], c, g,
                                                        1e-8, 0.0, 250, f), PARITY)


@pytest.mark.parametrize("depth", [2, 0])
def test_two_iteration_batch_equals_one_iteration_batch(ctx, depth):
    inst = _mixed_batch(8, EVEN)
    ctx.set_depth(depth)
    try:
        st2, res2, outs2 = _run(ctx, inst, rtol=1e-9, max_iters=200)
        assert ctx.stats()["depth"] == (depth or 4)
    finally:
        ctx.set_depth(0)
    ctx.set_depth(1)
    try:
        st1, res1, outs1 = _run(ctx, inst, rtol=1e-9, max_iters=200)
        assert ctx.stats()["depth"] == 1
    finally:
        ctx.set_depth(0)
    for r2, r1, o2, o1 in zip(res2, res1, outs2, outs1):
        if r2["iters"] == r1["iters"]:
            assert np.array_equal(o2, o1)
        else:
            say("borderline stop decision", r2["iters"], r1["iters"])
            assert abs(r2["iters"] - r1["iters"]) <= 1 and rel(o2, o1) <= 1e-9


def test_batch_rejects_bad_instances(ctx):
    inst = _mixed_batch(4)[:2]
    bad = dict(inst[0])
    bad["h"] = -1.0
    st, _, _ = _run(ctx, [inst[1], bad], raise_on_error=False)
    assert st == B.LX_EINVAL
    assert "instance 1" in ctx.last_error()


def test_full_256_instance_workload(lx):
    items = W.batched_instances()
    n_tot = sum(p.N for p, _ in items)
    say("256-instance workload", n_tot, "points")
    with lx.context(n_max=1 << 16, k_max=1) as ctx:
        args, outs, vs = [], [], []
        for i, (p, u0) in enumerate(items):
            rho = 2.0 / W.diffadv_cfl_step(p.D, p.vx, p.vy, p.dx, p.dy)
            c, g = shift_scale(rho)
            o = dev(np.zeros_like(u0))
            vs.append(u0)
            outs.append(o)
            args.append(dict(op=B.make_operator(p), v=dev(u0), out=o, l=0, h=p.h, c=c, gamma=g))
        st, res = ctx.phi_leja_batched(args, rtol=1e-8, max_iters=300)
    assert st == B.LX_OK
    iters = [r["iters"] for r in res]
    say("sweeps min/median/max", min(iters), int(np.median(iters)), max(iters))
    # every instance: the sum invariant of the exp action (the periodic
    # stencil conserves the sum and xi_0 = 2 is a node)
    for v, o in zip(vs, outs):
        ho = host(o)
        assert abs(ho.sum() - v.sum()) <= 1e-12 * np.abs(v).sum()
    # a sample against the oracle
    for i in range(0, 256, 37):
        p, u0 = items[i]
        A = lambda y, p=p: diffadv_apply(y, p.D, p.vx, p.vy, p.dx, p.dy)
        c, g = res[i]["c"], res[i]["gamma"]
        oracle_parity([host(outs[i])], [res[i]["iters"]],
                      lambda f, A=A, u0=u0, p=p, c=c, g=g: leja_phi(A, u0, [(0, 1.0, 1.0)], p.h, c, g, 1e-8, 0.0,
                                                                    300, f), PARITY)


def test_batch_graph_replays_match_eager_runs(ctx):
    """The captured pipeline (power iteration, coefficients, windows) replays
    bitwise what the eager launches compute.  With capture on, the first
    call of a layout runs eagerly and captures; later calls replay.  The
    tighter tolerance needs more windows than the looser call captured: its
    first call replays those and goes on eagerly (and captures again).
    Every replay is checked against the eager result, with the program's
    own eager work and synchronisations between the calls."""
    import torch
    inst = _mixed_batch(9, EVEN)
    say("batch graph replays")
    kws = [dict(power_iters=20, rtol=1e-6, max_iters=200), dict(power_iters=20, rtol=1e-10, max_iters=200),
           dict(power_iters=0, rtol=1e-8, max_iters=200)]
    ctx.set_batch_graphs(False)
    eager = [_run(ctx, inst, **kw) for kw in kws]
    ctx.set_batch_graphs(True)
    expect_replayed = [[0, 1, 1, 1], [1, 1, 1, 1], [0, 1, 1, 1]]
    for kw, (st0, res0, outs0), flags in zip(kws, eager, expect_replayed):
        assert st0 == B.LX_OK
        for k in range(4):
            st, res, outs = _run(ctx, inst, **kw)
            assert ctx.stats()["batch_graph"] == flags[k], (kw, k)
            assert st == st0 and [r["iters"] for r in res] == [r["iters"] for r in res0]
            assert all(np.array_equal(a, b) for a, b in zip(outs, outs0)), (kw, k)
            # the program's own eager work between replays
            q = inst[0]
            o = dev(np.zeros((q["ny"], q["nx"])))
            ctx.phi_leja(q["op"], dev(q["v"]), [o], [q["l"]], q["h"], q["c"], q["gamma"], rtol=1e-8,
                         max_iters=200, **({"u": dev(q["u"])} if q["u"] is not None else {}))
            torch.cuda.synchronize()
    # the eager result itself against the oracle (power iteration off)
    st0, res0, outs0 = eager[2]
    for q, r, o in zip(inst, res0, outs0):
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"],
                                              1e-8, 0.0, 200, f), PARITY)


@pytest.mark.parametrize("depth,th,ppw", [(4, 8, 4096), (4, 16, 32768), (2, 16, 8192), (1, 0, 4096)])
def test_batch_shapes_match_oracle(ctx, depth, th, ppw):
    """Every launch shape the batch tuner may pick (iterations per launch,
    tile rows, points per workgroup: several workgroups per instance)."""
    inst = _mixed_batch(10, [(256, 256, "da"), (96, 40, "da"), (130, 66, "da"), (512, 128, "da"), (64, 64, "da")])
    args_probe = [dict(op=q["op"], v=dev(q["v"]), out=dev(np.zeros((q["ny"], q["nx"]))), h=q["h"]) for q in inst]
    ctx.set_batch_shape(args_probe, depth, th, ppw)
    say("batch shape", depth, th, ppw)
    try:
        st, res, outs = _run(ctx, inst, rtol=1e-8, max_iters=200)
        assert ctx.stats()["depth"] == depth
    finally:
        ctx.set_batch_shape(args_probe)
    assert st == B.LX_OK
    for q, r, o in zip(inst, res, outs):
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"],
                                              1e-8, 0.0, 200, f), PARITY)


def test_batch_tuner_keeps_the_fastest_shape(ctx):
    inst = _mixed_batch(11, EVEN)
    args = [dict(op=q["op"], v=dev(q["v"]), out=dev(np.zeros((q["ny"], q["nx"]))), l=q["l"], h=q["h"], c=q["c"],
                 gamma=q["gamma"], **({"u": dev(q["u"])} if q["u"] is not None else {})) for q in inst]
    say("batch tuner")
    rows = ctx.tune_batched(args, rtol=1e-8, max_iters=200, repeats=1)
    # Burgers instances present: windows take 8-row tiles only
    assert {(r[0], r[1]) for r in rows} == {(4, 8), (2, 8), (2, 16), (1, 8)}
    assert all(r[3] > 0 for r in rows)
    best = min(rows, key=lambda r: r[3])
    st, res, outs = _run(ctx, inst, rtol=1e-8, max_iters=200)
    assert st == B.LX_OK and ctx.stats()["depth"] == best[0]
    ctx.set_batch_shape(args)
    for q, r, o in zip(inst, res, outs):
        oracle_parity([o], [r["iters"]],
                      lambda f, q=q: leja_phi(q["A"], q["v"], [(q["l"], 1.0, 1.0)], q["h"], q["c"], q["gamma"],
                                              1e-8, 0.0, 200, f), PARITY)
