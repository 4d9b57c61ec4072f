"""P5 (lambda schedule), P8 (loss closed forms), P9 (Adam first step),
all on the CPU oracle."""

import os

import numpy as np
import pytest
import torch

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_lambda_schedule_golden():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "lambda_schedule.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 6
    for ite, val in rows:
        assert oracle.lambda_at(int(ite)) == pytest.approx(float(val), rel=1e-12)
    assert oracle.lambda_at(3708) < 300.0 <= oracle.lambda_at(3709)


def _unit(rng, shape):
    n = rng.normal(size=(3,) + shape)
    return n / np.linalg.norm(n, axis=0, keepdims=True)


def test_loss_zero_at_target():
    rng = np.random.default_rng(0)
    Nt = _unit(rng, (6, 5))
    Dt = rng.uniform(1, 3, size=(6, 5))
    D = torch.tensor(Dt, requires_grad=True)
    N = torch.tensor(Nt, requires_grad=True)
    L = oracle.render_loss(D, N, Dt, Nt)
    assert float(L) == pytest.approx(0.0, abs=1e-12)
    L.backward()
    # |1 - N.N_hat| is ~1e-16 off zero; the other two terms are exactly 0 with sgn(0) = 0
    assert float(D.grad.abs().max()) == 0.0
    assert float(N.grad.abs().max()) <= 5.0 * np.abs(Nt).max() + 1e-12


def test_loss_scaled_normal_closed_form():
    rng = np.random.default_rng(1)
    Nt = _unit(rng, (4, 7))
    Dt = rng.uniform(1, 3, size=(4, 7))
    c = 0.6
    N = torch.tensor(c * Nt, requires_grad=True)
    D = torch.tensor(Dt + 0.25, requires_grad=True)
    a1, a2 = 5.0, 1.0
    L = oracle.render_loss(D, N, Dt, Nt)
    P = Dt.size
    expect = a1 * (1 - c) * P + a1 * (1 - c) * np.abs(Nt).sum() + a2 * 0.25 * P
    assert float(L) == pytest.approx(expect, rel=1e-12)
    L.backward()
    np.testing.assert_allclose(N.grad.numpy(), -a1 * (Nt + np.sign(Nt)), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(D.grad.numpy(), a2 * np.ones_like(Dt), rtol=0, atol=0)


def test_loss_terms_mask_and_mean():
    rng = np.random.default_rng(2)
    Nt = _unit(rng, (3, 3))
    N = _unit(rng, (3, 3))
    D = rng.uniform(size=(3, 3))
    Dt = rng.uniform(size=(3, 3))
    mask = np.zeros((3, 3))
    mask[1, 2] = 1
    t = oracle.loss_terms(D, N, Dt, Nt, mask=mask)
    assert float(t[2]) == pytest.approx(abs(D[1, 2] - Dt[1, 2]))
    assert float(t[0]) == pytest.approx(5 * abs(1 - (N[:, 1, 2] * Nt[:, 1, 2]).sum()))
    tm = oracle.loss_terms(D, N, Dt, Nt, reduction="mean")
    ts = oracle.loss_terms(D, N, Dt, Nt)
    for a, b in zip(tm, ts):
        assert float(a) == pytest.approx(float(b) / 9)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    theta = rng.normal(size=50)
    g = rng.normal(size=50) * 10 ** rng.uniform(-3, 3, size=50)
    th, m, v = oracle.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(th - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_second_step_and_clamp():
    theta = np.array([0.5, 1e-4 + 1e-7])
    g1 = np.array([1.0, 1.0])
    th, m, v = oracle.adam_step(theta, g1, np.zeros(2), np.zeros(2), 1, clamp_min=1e-4)
    assert th[1] == 1e-4
    g2 = np.array([-2.0, 0.5])
    th2, m2, v2 = oracle.adam_step(th, g2, m, v, 2)
    m_ref = 0.9 * 0.1 * g1 + 0.1 * g2
    v_ref = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    step = 1e-3 * (m_ref / (1 - 0.81)) / (np.sqrt(v_ref / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(th2, th - step, rtol=1e-12)
