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
