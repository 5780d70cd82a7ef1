"""Pins of the learned-potential oracle: reverse-mode gradient against central
finite differences; activation derivative; output scaling."""
import math

import numpy as np

from oracle import mlp_oracle as MO
from workloads.mlp_inputs import init_params, n_params


def test_param_count_matches_layout():
    assert n_params(6) == MO.n_params(6) == 34310


def test_dsilu_is_derivative():
    x = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (MO.silu(x + h) - MO.silu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - MO.dsilu(x))) < 1e-9


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    th = init_params(3).astype(np.float64)
    d = rng.uniform(1.0, 8.0, size=(12, 3))
    v = rng.uniform(0.0, 0.09, size=(12, 3))
    loss, g = MO.loss_and_grad(th, d, v, 3)
    idx = rng.choice(th.size, size=40, replace=False)
    idx = np.concatenate([idx, [0, 3 * 128, 3 * 128 + 128, th.size - 1]])   # W1, b1, W2, b4
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (MO.loss_and_grad(tp, d, v, 3)[0] - MO.loss_and_grad(tm, d, v, 3)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(fd)


def test_zero_last_layer_outputs_bias():
    th = init_params(6).astype(np.float64)
    n = th.size
    th[n - 6 - 128 * 6:n - 6] = 0.0
    th[n - 6:] = np.arange(6) * 0.5
    v = MO.potential(th, np.array([[2.0, 1.4, 3.0], [5.0, 2.0, 6.5]]), 6)
    assert np.allclose(v, MO.OUT_SCALE * np.arange(6) * 0.5)


def test_forward_of_a_hand_wired_network():
    """Sparse weights wired by hand: one path feature 2 -> hidden 5 -> hidden 7 ->
    hidden 9 -> every output, so the outputs follow from scalar arithmetic written
    out here (row-major [in][out] weights, SiLU on the three hidden layers only)."""
    n_out = 6
    th = np.zeros(MO.n_params(n_out))
    H = MO.HIDDEN
    o_w1, o_b1 = 0, 3 * H
    o_w2 = o_b1 + H
    o_b2 = o_w2 + H * H
    o_w3 = o_b2 + H
    o_b3 = o_w3 + H * H
    o_w4 = o_b3 + H
    o_b4 = o_w4 + H * n_out
    th[o_w1 + 2 * H + 5] = 1.5
    th[o_b1 + 5] = -0.25
    th[o_w2 + 5 * H + 7] = 2.0
    th[o_b2 + 7] = 0.5
    th[o_w3 + 7 * H + 9] = -1.0
    for k in range(n_out):
        th[o_w4 + 9 * n_out + k] = k + 1.0
        th[o_b4 + k] = 0.1 * k
    d = np.array([[2.0, 1.4, 3.0], [5.0, 2.0, 6.5], [1.0, 7.0, 0.7]])

    def s(x):
        return x / (1.0 + math.exp(-x))
    for row in range(d.shape[0]):
        f2 = (d[row, 2] - 4.0) / 3.0
        a3 = s(-s(2.0 * s(1.5 * f2 - 0.25) + 0.5))
        want = [0.1 * ((k + 1.0) * a3 + 0.1 * k) for k in range(n_out)]
        got = MO.potential(th, d[row:row + 1], n_out)[0]
        assert np.max(np.abs(got - np.array(want))) < 1e-15
