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
