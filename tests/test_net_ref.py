"""Pins of the warm-start network's CPU reference: its analytic gradient
against central finite differences (FP64), the zero padding at column ends,
and the bfloat16 rounding against the format's definition."""
import numpy as np
import pytest

import workloads as W
from oracle import net_ref as N


def _batch(seed):
    cols = [(9, 0.8, 3e-5, 1, 1.2, 4.2), (14, 0.9, 1e-6, 2, 0.7, 3.0), (6, 0.72, 1e-4, 1, 2.1, 5.5)]
    xs = [N.features(*c) for c in cols]
    rng = W.uniform_pm1(seed, sum(2 * c[0] for c in cols))
    tg, k = [], 0
    for c in cols:
        tg.append(0.3 * rng[k:k + 2 * c[0]].reshape(2, c[0]))
        k += 2 * c[0]
    return xs, tg


def test_parameter_count():
    assert N.n_params() == 8 * 5 * 64 + 64 + 4 * (64 * 5 * 64 + 64) + 64 * 5 * 2 + 2


def test_gradient_matches_central_differences():
    theta = N.init_params(11)
    theta = theta + 0.05 * W.uniform_pm1(12, theta.size)  # nonzero biases too
    xs, tg = _batch(13)
    L, g = N.loss_and_grad(theta, xs, tg)
    idx = np.concatenate([np.arange(0, 40, 7), np.arange(2560, 2660, 13),
                          np.arange(N.n_params() - 700, N.n_params(), 37)])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (N.loss_and_grad(tp, xs, tg)[0] - N.loss_and_grad(tm, xs, tg)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_columns_do_not_see_each_other():
    """The zero padding makes a column's output independent of where it sits
    in a batch: evaluating the columns alone or together gives the same loss."""
    theta = N.init_params(3)
    xs, tg = _batch(4)
    L_all, g_all = N.loss_and_grad(theta, xs, tg)
    parts = [N.loss_and_grad(theta, [x], [t]) for x, t in zip(xs, tg)]
    w = np.array([x.shape[1] for x in xs], dtype=float)
    assert L_all == pytest.approx((np.array([p[0] for p in parts]) * w).sum() / w.sum(), rel=1e-12)


def test_bf16_rounding():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to even (1.0)
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.1415926, -2.5e-3])
    r = N.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6
    assert abs(r[3] - np.pi) < 2 ** -7 * 4 and abs(r[4] + 2.5e-3) < 2.5e-3 * 2 ** -8


def test_adam_with_a_constant_gradient_moves_by_lr_every_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves a parameter by lr g / (|g| + eps)."""
    g = np.array([3.0, -0.25, 1e-3, 0.0])
    theta, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    lr = 1e-2
    for t in range(1, 6):
        theta, m, v = N.adam_step(theta, g, m, v, t, lr)
        np.testing.assert_allclose(theta, -t * lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_interface_channels():
    """The two interface channels are zero at the lever-rule height, odd
    about it, and saturate at +-1 at 128 and 16 nodes away."""
    x = N.features(300, 0.8, 1e-5, 1, 1.3, 100.0)
    y = np.arange(300) + 0.5
    assert np.all(np.sign(x[6]) == np.sign(y - 100.0)) and np.all(np.sign(x[7]) == np.sign(y - 100.0))
    assert abs(x[6][99]) < 1 / 128 and abs(x[7][100]) == 0.5 / 16
    assert x[6][0] == -99.5 / 128 and x[6][-1] == 1.0 and x[7][0] == -1.0 and x[7][-1] == 1.0
