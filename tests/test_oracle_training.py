"""Pins of the reference's student loss, gradient and optimizer step."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import em_volume
from synth.nets import NET_S, he_normal_params, random_bias_params

SMALL_S = [{"kind": "conv", "k": 3, "cin": 1, "cout": 3, "act": "relu"},
           {"kind": "conv", "k": 3, "cin": 3, "cout": 2, "act": "relu"},
           {"kind": "conv", "k": 1, "cin": 2, "cout": 1, "act": "sigmoid"}]


def _loss_only(patches, teacher, net, p):
    return oracle.student_loss_grad(patches, teacher, net, p)[0]


def test_loss_matches_bce_definition():
    # L = mean over outputs of -[t log s + (1-t) log(1-s)], s = sigmoid(z).
    rng = np.random.default_rng(0)
    patches = rng.integers(0, 256, size=(2, 12, 12), dtype=np.uint8)
    p = random_bias_params(SMALL_S, 1, 2, sigma=0.3)
    z = oracle.forward(patches, SMALL_S, p, logits=True)
    t = rng.uniform(0, 1, size=z.shape)
    s = 1.0 / (1.0 + np.exp(-z))
    bce = -(t * np.log(s) + (1 - t) * np.log1p(-s)).mean()
    loss, _ = oracle.student_loss_grad(patches, t, SMALL_S, p)
    assert loss == pytest.approx(bce, rel=1e-12)


def test_head_gradient_closed_form():
    # dL/db_head = mean(sigmoid(z) - t) exactly (bias enters every logit once).
    rng = np.random.default_rng(1)
    patches = rng.integers(0, 256, size=(3, 10, 10), dtype=np.uint8)
    p = random_bias_params(SMALL_S, 3, 4, sigma=0.3)
    z = oracle.forward(patches, SMALL_S, p, logits=True)
    t = rng.uniform(0, 1, size=z.shape)
    _, g = oracle.student_loss_grad(patches, t, SMALL_S, p)
    assert g[-1] == pytest.approx((1.0 / (1.0 + np.exp(-z)) - t).mean(), rel=1e-12)


@pytest.mark.parametrize("net,seed", [(SMALL_S, 5), (NET_S, 300)])
def test_gradient_central_differences(net, seed):
    rng = np.random.default_rng(seed)
    P = 14 if net is SMALL_S else 16
    patches = em_volume(seed, 2, P, P)
    p = random_bias_params(net, seed, seed + 1, sigma=0.2)
    R = oracle.radius(net)
    t = rng.uniform(0, 1, size=(2, P - R, P - R))
    _, g = oracle.student_loss_grad(patches, t, net, p)
    idx = np.arange(p.size) if p.size < 120 else rng.choice(p.size, 120, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (_loss_only(patches, t, net, pp) - _loss_only(patches, t, net, pm)) / (2 * h)
        # a ReLU kink inside [p-h, p+h] is the only way this can fail
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_step_one_closed_form():
    # With m = v = 0 at t = 1: m_hat = g, v_hat = g^2, step = -lr g / (|g| + eps).
    rng = np.random.default_rng(2)
    g = rng.normal(size=50) * 10.0 ** rng.integers(-6, 2, size=50)
    th = rng.normal(size=50)
    th0 = th.copy()
    m, v = np.zeros(50), np.zeros(50)
    oracle.adam(th, m, v, g, 1, lr=1e-3)
    assert np.allclose(th, th0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_matches_recurrence_over_steps():
    rng = np.random.default_rng(3)
    th, m, v = rng.normal(size=8), np.zeros(8), np.zeros(8)
    th2, m2, v2 = th.copy(), m.copy(), v.copy()
    for t in range(1, 6):
        g = rng.normal(size=8)
        oracle.adam(th, m, v, g, t, lr=0.01, b1=0.8, b2=0.9, eps=1e-6)
        m2 = 0.8 * m2 + 0.2 * g
        v2 = 0.9 * v2 + 0.1 * g * g
        th2 = th2 - 0.01 * (m2 / (1 - 0.8 ** t)) / (np.sqrt(v2 / (1 - 0.9 ** t)) + 1e-6)
    assert np.allclose(th, th2, rtol=1e-14, atol=1e-15)


def test_calibration_file_is_current():
    from oracle import calibrate
    stored = json.load(open(calibrate.OUT))
    fresh = calibrate.compute()
    for name in ("A", "B"):
        assert stored[name]["head_bias"] == pytest.approx(fresh[name]["head_bias"], abs=1e-12)
    for a, b in zip(stored["B"]["act_scales"], fresh["B"]["act_scales"]):
        assert (a is None and b is None) or a == pytest.approx(b, rel=1e-12)


def test_calibrated_head_bias_splits_map():
    from oracle import calibrate
    from synth.nets import calibrated_params, NET_B
    img = calibrate.calibration_slice()
    prob = oracle.forward(img[None], NET_B, calibrated_params("B"))
    frac = (prob >= 0.5).mean()
    assert 0.49 <= frac <= 0.51
