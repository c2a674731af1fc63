"""The learned spectral-bound / budget path on the GPU.

Acceptance is decided by the Leja stop rule itself: an instance whose
predicted interval and budget do not lead to convergence is solved again by
the plain method.  The tests check (1) that a small predictor trained from
records of the plain method gives converged results that agree with the
plain method, (2) that a predictor that is always wrong sends every
instance down the fallback, whose results are then those of the plain
batched method bit for bit, and (3) that the committed predictor accepts
most instances of its evaluation distribution and saves sweeps.
"""
import os

import numpy as np
import pytest

from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import learned as L
from oracle.mlp import N_PARAMS
from tests.gpu_helpers import host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=1 << 16, k_max=1)
    yield c
    c.close()


def _items(count, seed0, sizes=(64,)):
    from paper_2310_08344_amd import workloads as W
    return [W.learned_instance(i, seed0, sizes) for i in range(count)]


def test_small_trained_predictor_agrees_with_plain(ctx):
    say("learned: records 192 x 64^2")
    X, Y, K = L.generate_records(ctx, 192, 100000, batch=96, sizes=(64,))
    assert X.shape[0] >= 180 and np.all(np.isfinite(X)) and np.all(np.isfinite(Y))
    say("learned: train 400 steps")
    p, summary = L.train_predictor(ctx, X, Y, steps=400, batch=64, lr=3e-3)
    assert np.isfinite(summary["val_rmse_log_rho"])
    say("learned: calibrate on 64")
    margin_s, cal = L.calibrate_budget(ctx, p, summary["margin_log_rho"], count=64, sizes=(64,))
    assert np.isfinite(margin_s) and cal["calibration_instances"] == 64
    items = _items(24, 700000)
    args, keep = L._instance_args(items, "cuda:0")
    import torch
    plain_out = [torch.empty_like(a["out"]) for a in args]
    say("learned: plain batched 24")
    res_p = L.solve_plain(ctx, [dict(a, out=o) for a, o in zip(args, plain_out)])
    say("learned: learned batched 24")
    res_l, fb = L.solve_learned(ctx, p, args, summary["margin_log_rho"], margin_s)
    say("accepted", 24 - len(fb), "fallbacks", len(fb))
    for i, (a, o, rp, rl) in enumerate(zip(args, plain_out, res_p, res_l)):
        assert rp["status"] == B.LX_OK and rl["status"] == B.LX_OK, (i, rp, rl)
        assert rel(host(a["out"]), host(o)) <= 1e-6, i


def test_wrong_predictor_falls_back_to_plain_bit_for_bit(ctx):
    p = ctx.predictor()
    s = np.zeros(3 * N_PARAMS + 21, dtype=np.float32)
    s[3 * N_PARAMS + 8:3 * N_PARAMS + 16] = 1.0          # std_x
    s[3 * N_PARAMS + 16] = np.log(1e-6)                   # mean_y: rho = 1e-6 ...
    s[3 * N_PARAMS + 17] = 0.0                            # ... and a budget of 1 (+2) sweeps
    s[3 * N_PARAMS + 18:3 * N_PARAMS + 20] = 1.0          # std_y
    p.set_state(s)
    items = _items(16, 710000, sizes=(64, 128))
    args, keep = L._instance_args(items, "cuda:0")
    import torch
    plain_out = [torch.empty_like(a["out"]) for a in args]
    say("learned: forced fallback 16")
    res_p = L.solve_plain(ctx, [dict(a, out=o) for a, o in zip(args, plain_out)])
    res_l, fb = L.solve_learned(ctx, p, args, 0.0, 0.0)
    assert fb == list(range(16))
    for a, o, rp, rl in zip(args, plain_out, res_p, res_l):
        assert rl["status"] == B.LX_OK and rl["iters"] == rp["iters"]
        assert torch.equal(a["out"], o)


@pytest.mark.skipif(not os.path.exists(L.PREDICTOR_FILE), reason="no committed predictor")
def test_committed_predictor_saves_sweeps(ctx):
    p, margins, meta = L.load_predictor(ctx)
    items = _items(64, 900000, sizes=(128,))
    args, keep = L._instance_args(items, "cuda:0")
    import torch
    plain_out = [torch.empty_like(a["out"]) for a in args]
    say("learned: committed predictor on 64 x 128^2")
    res_p = L.solve_plain(ctx, [dict(a, out=o) for a, o in zip(args, plain_out)])
    res_l, fb = L.solve_learned(ctx, p, args, *margins)
    assert all(r["status"] == B.LX_OK for r in res_l)
    assert len(fb) <= 64 // 10, fb
    sweeps_p = sum(r["iters"] for r in res_p) + L.POWER_ITERS * 64
    sweeps_l = sum(r["iters"] for r in res_l) + L.POWER_ITERS * len(fb)
    say("sweeps plain", sweeps_p, "learned", sweeps_l)
    assert sweeps_l < sweeps_p
    for a, o in zip(args, plain_out):
        assert rel(host(a["out"]), host(o)) <= 1e-6


def _oracle_apply(prm, u):
    from oracle.operators import make_apply
    return make_apply(prm, u)


def _exact(prm, u, v, l, A):
    """phi_l(hA)v without the library: the Fourier solution for
    diffusion-advection; for the Burgers Jacobian (not diagonalised by the
    FFT) the oracle's own Leja loop at rtol 1e-13 with the closed-form
    Gershgorin interval, which lies outside every eigenvalue."""
    from oracle.exact import phi_fft
    from oracle.phi_action import leja_phi, shift_scale
    from paper_2310_08344_amd import workloads as W
    if prm.kind == W.DIFFADV:
        return phi_fft(v, l, prm.h, prm.D, prm.vx, prm.vy, prm.dx, prm.dy)
    umax = float(np.max(np.abs(u)))
    rho = 2.0 / W.burgers_cfl_step(prm.nu, umax, prm.dx, prm.dy)
    c, g = shift_scale(rho)
    r = leja_phi(A, v, [(l, 1.0, 1.0)], prm.h, c, g, 1e-13, 0.0, 600)
    assert r.status == "ok"
    return r.p[0]


@pytest.mark.skipif(not os.path.exists(L.PREDICTOR_FILE), reason="no committed predictor")
@pytest.mark.parametrize("size,seed0", [(64, 720000), (128, 730000)])
def test_learned_solves_match_oracle_and_exact_solution(ctx, size, seed0):
    """Every instance of a learned batch (the committed predictor; half
    diffusion-advection, half Burgers), accepted or fallen back, against
    (1) the oracle's Leja loop run with the shift and scale the GPU used and
    its own stop rule at the same tolerance, at 1e-10 (a flipped borderline
    stop is compared at the GPU's count); (2) the exact phi_l(hA)v at ten
    times the tolerance (the reading for several correct results); and the
    plain batched method's solve of the same instance against the same
    exact solution."""
    import torch

    from oracle.phi_action import leja_phi
    from tests.gpu_helpers import oracle_parity
    p, margins, meta = L.load_predictor(ctx)
    items = _items(12, seed0, sizes=(size,))
    args, keep = L._instance_args(items, "cuda:0")
    plain_out = [torch.empty_like(a["out"]) for a in args]
    say("learned vs oracle and exact", size, seed0)
    res_l, fb = L.solve_learned(ctx, p, args, *margins)
    res_p = L.solve_plain(ctx, [dict(a, out=o) for a, o in zip(args, plain_out)])
    worst = [0.0, 0.0, 0.0]
    for i, ((prm, u, v), a, rl, rp, op_) in enumerate(zip(items, args, res_l, res_p, plain_out)):
        assert rl["status"] == B.LX_OK and rp["status"] == B.LX_OK, (i, rl, rp)
        l = prm.meta["l"]
        A = _oracle_apply(prm, u)
        got = host(a["out"])
        mi = rl["iters"] + 8
        _, errs, flipped = oracle_parity(
            [got], [rl["iters"]],
            lambda f: leja_phi(A, v, [(l, 1.0, 1.0)], prm.h, rl["c"], rl["gamma"], L.RTOL, 0.0, mi, f), 1e-10)
        ex = _exact(prm, u, v, l, A)
        e_l, e_p = rel(got, ex), rel(host(op_), ex)
        say(f"instance {i} ({prm.kind}, l={l}, fallback={rl['fallback']}): oracle {errs[0]:.2e}, "
            f"exact learned {e_l:.2e} plain {e_p:.2e}, sweeps learned {rl['iters']} plain {rp['iters']}")
        worst = [max(worst[0], errs[0]), max(worst[1], e_l), max(worst[2], e_p)]
        assert e_l <= 10 * L.RTOL and e_p <= 10 * L.RTOL, (i, e_l, e_p)
    say("worst: oracle parity", worst[0], "exact learned", worst[1], "exact plain", worst[2])
