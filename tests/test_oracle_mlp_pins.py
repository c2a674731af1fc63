"""Pins of the oracle MLP against facts fixed outside it.

* bfloat16 rounding: exactly representable values, ties to even, the
  largest rounding error of 2^-9 relative.
* Backward pass: central finite differences of the loss (rounding off).
* Adam: the first step from zero moments moves each parameter by lr times
  the sign of its gradient (up to eps), the closed form of bias-corrected
  Adam at t = 1.
* A linear target is fitted (training decreases the loss by orders of
  magnitude).
"""
import numpy as np

from oracle.mlp import N_PARAMS, adam_step, bf16, forward, loss_and_grad, pack, unpack


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3.0 * 2.0**-8, 1.0 + 2.0**-9, -2.5, 0.0, 3.0e-5])
    r = bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie between 1 and 1+2^-7 goes to the even 1
    assert r[2] == 1.0 + 2.0**-6            # tie between 1+2^-7 and 1+2^-6 goes to even 1+2^-6...
    assert r[3] == 1.0
    assert r[4] == -2.5 and r[5] == 0.0
    rng = np.random.default_rng(0)
    y = rng.standard_normal(10000) * 10.0
    assert np.max(np.abs(bf16(y) - y) / np.abs(y)) <= 2.0**-8 + 1e-12


def _params(seed=1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N_PARAMS) * 0.3


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((17, 8))
    T = rng.standard_normal((17, 2))
    th = _params()
    loss, g = loss_and_grad(th, X, T, round_bf16=False)
    e = 1e-6
    idx = rng.choice(N_PARAMS, 60, replace=False)
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += e
        tm[i] -= e
        fd = (loss_and_grad(tp, X, T, False)[0] - loss_and_grad(tm, X, T, False)[0]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_pack_unpack_roundtrip():
    th = _params(3)
    assert np.array_equal(pack(unpack(th)), th)
    assert N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.default_rng(4)
    th = _params(5)
    g = rng.standard_normal(N_PARAMS)
    new, m, v = adam_step(th, g, np.zeros(N_PARAMS), np.zeros(N_PARAMS), 1, 1e-3)
    step = th - new
    assert np.allclose(step, 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_fits_a_linear_target():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((512, 8))
    A = rng.standard_normal((8, 2))
    T = X @ A
    th = _params(7) * 0.5
    m = np.zeros(N_PARAMS)
    v = np.zeros(N_PARAMS)
    l0 = loss_and_grad(th, X, T)[0]
    for t in range(1, 801):
        loss, g = loss_and_grad(th, X, T)
        th, m, v = adam_step(th, g, m, v, t, 3e-3)
    assert loss < 0.02 * l0
    Y, _ = forward(th, X)
    assert Y.shape == (512, 2)
