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


def test_adam_constant_gradient_gives_unbiased_moments_at_every_step():
    """With the same gradient g at every step, the bias-corrected moments
    equal g and g^2 exactly for every t (Kingma and Ba 2015, Sec. 3), so
    every step moves by lr * g / (|g| + eps): a wrong decay rate or a
    missing or misplaced bias correction in either moment breaks this at
    t >= 2."""
    rng = np.random.default_rng(11)
    g = rng.standard_normal(N_PARAMS) * np.exp(rng.uniform(-3, 3, N_PARAMS))
    th = _params(12)
    m = np.zeros(N_PARAMS)
    v = np.zeros(N_PARAMS)
    lr = 2e-3
    for t in range(1, 40):
        new, m, v = adam_step(th, g, m, v, t, lr, beta1=0.8, beta2=0.99)
        assert np.allclose(th - new, lr * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=0.0), t
        th = new


def test_adam_moments_are_normalised_exponential_averages():
    """After gradients g_1..g_t, the bias-corrected first moment is the
    average of the g_i weighted by beta1^(t-i) and the second the average of
    the g_i^2 weighted by beta2^(t-i) (the weights sum to
    (1 - beta^t) / (1 - beta), which the correction divides out).  Checked
    with exact rational weights on changing gradients for t = 1..6."""
    from fractions import Fraction as Fr

    b1, b2, lr = Fr(9, 10), Fr(999, 1000), 1e-2
    gs = [Fr(3, 2), Fr(-1, 2), Fr(1, 4), Fr(2), Fr(-3), Fr(1, 8)]
    th = np.array([0.5])
    m = np.zeros(1)
    v = np.zeros(1)
    for t in range(1, len(gs) + 1):
        new, m, v = adam_step(th, np.array([float(gs[t - 1])]), m, v, t, lr, beta1=float(b1), beta2=float(b2),
                              eps=0.0)
        w1 = [b1 ** (t - i) for i in range(1, t + 1)]
        w2 = [b2 ** (t - i) for i in range(1, t + 1)]
        mhat = sum(w * g for w, g in zip(w1, gs)) / sum(w1)
        vhat = sum(w * g * g for w, g in zip(w2, gs)) / sum(w2)
        expect = lr * float(mhat) / float(vhat) ** 0.5
        assert abs((th - new)[0] - expect) <= 1e-12 * abs(expect), (t, (th - new)[0], expect)
        th = new


def test_adam_step_is_invariant_to_gradient_scale():
    """With eps = 0 the update does not change when every gradient is
    multiplied by the same positive constant (the second moment is of g^2
    and enters through its square root)."""
    rng = np.random.default_rng(13)
    gs = rng.standard_normal((5, N_PARAMS))
    runs = []
    for s in (1.0, 1e-3, 37.0):
        th = _params(14)
        m = np.zeros(N_PARAMS)
        v = np.zeros(N_PARAMS)
        for t in range(1, 6):
            th, m, v = adam_step(th, s * gs[t - 1], m, v, t, 1e-3, eps=0.0)
        runs.append(th)
    assert np.allclose(runs[0], runs[1], rtol=1e-12, atol=1e-15)
    assert np.allclose(runs[0], runs[2], rtol=1e-12, atol=1e-15)
