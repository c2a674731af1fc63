"""GPU parity of the predictor MLP kernels (forward, backward, Adam,
inference) and of the feature kernel against the FP64 oracle, through the
C ABI.

Tolerances: the GPU computes in float32 with bfloat16 activations; the
oracle computes in float64 with the same two roundings of the activations.
A bfloat16 rounding decision can flip when the float32 and float64
pre-activations straddle a tie, so gradients and parameters are compared
in relative L2 norm (1e-4), not element by element.
"""
import numpy as np
import pytest

from oracle.mlp import N_PARAMS, adam_step, forward, loss_and_grad
from paper_2310_08344_amd import binding as B
from tests.gpu_helpers import dev, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lx):
    c = lx.context(n_max=1 << 16, k_max=1)
    yield c
    c.close()


def _f32(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


def _state(theta, mx, sx, my, sy, t=0):
    s = np.zeros(3 * N_PARAMS + 21, dtype=np.float32)
    s[:N_PARAMS] = theta
    s[3 * N_PARAMS:3 * N_PARAMS + 8] = mx
    s[3 * N_PARAMS + 8:3 * N_PARAMS + 16] = sx
    s[3 * N_PARAMS + 16:3 * N_PARAMS + 18] = my
    s[3 * N_PARAMS + 18:3 * N_PARAMS + 20] = sy
    s[-1] = t
    return s


def _problem(seed, n=300):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(N_PARAMS) * 0.2).astype(np.float32)
    X = rng.standard_normal((n, 8)) * 3.0 + 1.0
    T = rng.standard_normal((n, 2)) * 2.0 - 0.5
    mx, sx = X.mean(axis=0), X.std(axis=0)
    my, sy = T.mean(axis=0), T.std(axis=0)
    return theta, X.astype(np.float32), T.astype(np.float32), mx, sx, my, sy


def _std(X, T, mx, sx, my, sy):
    f = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Xs = (f(X) - f(mx).astype(np.float32)) / f(sx).astype(np.float32)
    Ts = (f(T) - f(my).astype(np.float32)) / f(sy).astype(np.float32)
    return Xs, Ts


def test_gradient_matches_oracle(ctx):
    theta, X, T, mx, sx, my, sy = _problem(0)
    p = ctx.predictor()
    p.set_state(_state(theta, mx, sx, my, sy))
    say("mlp gradient")
    loss, g = p.gradient(_f32(X), _f32(T))
    Xs, Ts = _std(X, T, mx, sx, my, sy)
    lo, go = loss_and_grad(theta.astype(np.float64), Xs, Ts)
    assert abs(loss - lo) <= 1e-5 * lo
    assert rel(g, go) <= 1e-4


def test_adam_training_matches_oracle(ctx):
    theta, X, T, mx, sx, my, sy = _problem(1)
    p = ctx.predictor()
    p.set_state(_state(theta, mx, sx, my, sy))
    steps, batch, lr = 10, 64, 1e-3
    order = np.random.default_rng(2).integers(0, X.shape[0], steps * batch)
    say("mlp adam")
    p.train(_f32(X), _f32(T), steps, batch, lr, order=order)
    got = p.get_state()
    Xs, Ts = _std(X, T, mx, sx, my, sy)
    th = theta.astype(np.float64)
    m = np.zeros(N_PARAMS)
    v = np.zeros(N_PARAMS)
    for k in range(steps):
        ix = order[k * batch:(k + 1) * batch]
        _, g = loss_and_grad(th, Xs[ix], Ts[ix])
        th, m, v = adam_step(th, g, m, v, k + 1, lr)
    assert rel(got[:N_PARAMS], th) <= 1e-4
    assert rel(got[N_PARAMS:2 * N_PARAMS], m) <= 1e-3
    assert got[-1] == steps


def test_inference_matches_oracle(ctx):
    theta, X, T, mx, sx, my, sy = _problem(3)
    p = ctx.predictor()
    p.set_state(_state(theta, mx, sx, my, sy))
    import torch
    out = torch.zeros(X.shape[0], 2, dtype=torch.float32, device="cuda:0")
    p.infer(_f32(X), out)
    torch.cuda.synchronize()
    Xs, _ = _std(X, T, mx, sx, my, sy)
    Y, _ = forward(theta.astype(np.float64), Xs)
    Y = Y * np.asarray(sy, dtype=np.float32) + np.asarray(my, dtype=np.float32)
    assert rel(host(out), Y) <= 1e-4


def test_save_load_roundtrip(ctx, tmp_path):
    theta, X, T, mx, sx, my, sy = _problem(4)
    p = ctx.predictor(seed=7)
    p.set_state(_state(theta, mx, sx, my, sy, t=5))
    p.train(_f32(X), _f32(T), 3, 32, 1e-3, seed=1)
    f = tmp_path / "pred.bin"
    p.save(f)
    q = ctx.predictor(seed=8)
    q.load(f)
    assert np.array_equal(p.get_state(), q.get_state())


def test_features_match_numpy(ctx):
    import torch
    rng = np.random.default_rng(5)
    inst, ref = [], []
    for i, (nx, ny, kind) in enumerate([(64, 64, "da"), (96, 40, "bu"), (33, 17, "da")]):
        v = rng.standard_normal((ny, nx)) * (i + 1)
        u = rng.standard_normal((ny, nx)) + 0.5
        h = 1e-4 * (i + 1)
        if kind == "da":
            op = B.make_operator(kind=B.LX_OP_DIFFADV2D, nx=nx, ny=ny, D=0.7, vx=-1.5, vy=2.0)
            inst.append(dict(op=op, v=dev(v), h=h, l=i))
            w = v
            ref.append([np.log(0.7), np.log(np.hypot(-1.5, 2.0) + 1e-3), np.arctan2(2.0, -1.5), np.log(1 / nx),
                        np.log(h), np.log(np.sqrt(np.mean(w * w))), np.log(np.max(np.abs(w))), i])
        else:
            op = B.make_operator(kind=B.LX_OP_BURGERS2D, nx=nx, ny=ny, nu=3e-3)
            inst.append(dict(op=op, v=dev(v), u=dev(u), h=h, l=i))
            w = u
            ref.append([np.log(3e-3), np.log(np.sqrt(2) * np.max(np.abs(w)) + 1e-3), np.pi / 4, np.log(1 / nx),
                        np.log(h), np.log(np.sqrt(np.mean(w * w))), np.log(np.max(np.abs(w))), i])
    out = torch.zeros(3, 8, dtype=torch.float32, device="cuda:0")
    ctx.features(inst, out)
    torch.cuda.synchronize()
    assert np.allclose(host(out), np.array(ref), rtol=1e-6, atol=1e-6)
