"""Pins of the rank-predictor oracle (CPU): finite differences for the gradient, closed forms
for the pinball loss and for a network with zero weights, and the parameter layout."""
import numpy as np
import pytest

from oracle import rank_mlp as rm


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 16)) * 2 + 1
    p = rm.init(x, seed)
    y = rm.forward(p, x)
    # targets well away from the predictions, so no sample sits on the kink of the pinball loss
    t = y + np.where(rng.random(n) < 0.5, -1.0, 1.0) * rng.uniform(0.5, 2.0, n)
    return p, x, t


def test_pinball_closed_form():
    y = np.array([0.0, 0.0, 1.0])
    t = np.array([1.0, -1.0, 1.0])
    # r = t - y = (1, -1, 0): tau * 1 + (1 - tau) * 1 + 0
    assert rm.pinball(y, t, 0.9) == pytest.approx(0.9 + 0.1)
    assert rm.pinball(y, t, 0.5) == pytest.approx(1.0)


def test_zero_weights_give_constant_output():
    x = np.random.default_rng(1).standard_normal((7, 16))
    d = rm.unpack(rm.init(x, 1))
    for k in ("W1", "W2", "W3", "b1", "b2"):
        d[k] = np.zeros_like(d[k])
    d["b3"] = 0.37
    p = rm.pack(d)
    assert np.allclose(rm.forward(p, x), 0.37)
    g = rm.grad(p, x, np.full(7, 1.37), 0.9)   # r = +1 everywhere: dL/db3 = -tau per sample
    assert rm.unpack(g)["b3"] == pytest.approx(-0.9 * 7)
    assert np.allclose(rm.unpack(g)["W3"], 0.0)   # h2 = tanh(0) = 0


def test_layout_round_trip_and_size():
    p = np.arange(rm.N_PARAM, dtype=float)
    assert rm.N_PARAM == 16 + 16 + 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1
    assert np.array_equal(rm.pack(rm.unpack(p)), p)
    assert rm.unpack(p)["W1"][2, 3] == 32 + 2 * 16 + 3


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    p, x, t = _data(seed)
    tau = 0.9
    g = rm.grad(p, x, t, tau)
    rng = np.random.default_rng(seed + 10)
    idx = np.concatenate([rng.choice(np.arange(32, rm.N_PARAM), 60, replace=False), [rm.N_PARAM - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros(rm.N_PARAM)
        e[i] = h
        fd = (rm.loss(p + e, x, t, tau) - rm.loss(p - e, x, t, tau)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i
    assert np.all(g[:32] == 0)


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected moments are g and g^2, so every trained
    entry moves by -lr g / (|g| + eps); the normalisation entries do not move."""
    rng = np.random.default_rng(3)
    p = rng.standard_normal(rm.N_PARAM)
    g = rng.standard_normal(rm.N_PARAM) * np.logspace(-3, 2, rm.N_PARAM)
    lr = 0.05
    p1, m, v = rm.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    assert np.array_equal(p1[:32], p[:32])
    assert np.allclose(p1[32:] - p[32:], -lr * g[32:] / (np.abs(g[32:]) + 1e-8), rtol=1e-12, atol=0)


def test_adam_two_steps_by_hand():
    """g = 2 then g = -1 on one weight, lr = 0.01, worked by hand:
    step 1: m = 0.2, v = 0.004, corrected 2 and 4 -> move -0.01 * 2 / (2 + 1e-8);
    step 2: m = 0.18 - 0.1 = 0.08, v = 0.003996 + 0.001 = 0.004996,
            corrected 0.08 / 0.19 and 0.004996 / 0.001999 -> move -0.01 * 0.421052... / 1.580901..."""
    i = 40
    p = np.zeros(rm.N_PARAM)
    m = np.zeros(rm.N_PARAM)
    v = np.zeros(rm.N_PARAM)
    g = np.zeros(rm.N_PARAM)
    g[i] = 2.0
    p, m, v = rm.adam_step(p, g, m, v, 1, 0.01)
    assert p[i] == pytest.approx(-0.02 / (2.0 + 1e-8), rel=1e-14)
    g[i] = -1.0
    p, m, v = rm.adam_step(p, g, m, v, 2, 0.01)
    assert m[i] == pytest.approx(0.08, rel=1e-14)
    assert v[i] == pytest.approx(0.004996, rel=1e-13)
    step2 = 0.01 * 0.42105263157894737 / (1.5809015228066567 + 1e-8)
    assert p[i] == pytest.approx(-0.02 / (2.0 + 1e-8) - step2, rel=1e-12)
    assert np.count_nonzero(p) == 1


def test_adam_invariant_to_gradient_scale():
    """Adam's step does not change when every gradient of a sequence is multiplied by one positive
    constant (up to eps), a property a missing square root or mismatched moment rates break."""
    rng = np.random.default_rng(4)
    p = rng.standard_normal(rm.N_PARAM)
    gs = [np.where(rng.random(rm.N_PARAM) < 0.5, -1.0, 1.0) * (0.5 + rng.random(rm.N_PARAM)) for _ in range(4)]
    a = (p, np.zeros_like(p), np.zeros_like(p))
    b = (p, np.zeros_like(p), np.zeros_like(p))
    for step, g in enumerate(gs, 1):
        a = rm.adam_step(a[0], g, a[1], a[2], step, 1e-3)
        b = rm.adam_step(b[0], 1e3 * g, b[1], b[2], step, 1e-3)
    assert np.abs(a[0] - p).max() > 1e-3
    assert np.abs(a[0] - b[0]).max() < 1e-9


def test_train_lowers_the_loss():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((300, 16))
    t = rm.forward(rm.init(x, 9), x)
    p0 = rm.init(x, 2)
    p1, hist = rm.train(p0, x, t, 0.9, 150, 3e-3)
    assert hist[0] == pytest.approx(rm.loss(p0, x, t, 0.9) / len(t))
    assert rm.loss(p1, x, t, 0.9) / len(t) < 0.5 * hist[0]
