"""Pins of the learned-initializer oracle: bfloat16 rounding on values fixed
by the format, max-pool against a loop, proposal decoding and plane
descriptors in closed form, the set loss on constructed matches, and the
reverse-mode gradient of the whole composition against central differences."""

import math

import numpy as np
import pytest
import torch

from oracle import initnet as net

F64 = torch.float64


def test_bf16_rounding_fixed_values():
    x = torch.tensor([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e38, 1e-40], dtype=F64)
    y = net.bf16(x)
    assert y[0] == 1.0
    assert y[1] == 1.0                    # halfway: ties to even
    assert y[2] == 1 + 2 ** -6            # halfway: ties to even (up)
    assert y[3] == 1 + 2 ** -7            # representable
    assert y[4] == -2.5
    assert float(y[5]) == round(3.0e38 / 2 ** 120) * 2.0 ** 120   # spacing 2^120 near 3e38
    assert abs(float(y[6])) < 1e-39


def test_pool_max_matches_loop():
    rng = np.random.default_rng(0)
    h = torch.tensor(rng.integers(0, 5, size=(2, 9, 4)).astype(np.float64))
    g, arg = net.pool_max(h)
    for b in range(2):
        for c in range(4):
            col = [float(h[b, n, c]) for n in range(9)]
            m = max(col)
            assert g[b, c] == m
            assert arg[b, c] == col.index(m)


def test_decode_and_descriptors_closed_form():
    out = torch.zeros(1, 2 * 12, dtype=F64)
    out[0, 12 + 3:12 + 7] = torch.tensor([-1.0, 0.0, 0.0, 1.0])   # quat (0, 0, 0, 1): 180 deg about z
    out[0, 12 + 7:12 + 11] = torch.tensor([2.0, 0.0, -1.0, 3.0])
    c, q, r, s = net.decode(out)
    assert torch.equal(c[0, 0], torch.zeros(3, dtype=F64))
    assert torch.allclose(q[0, 0], torch.tensor([1.0, 0, 0, 0], dtype=F64))
    assert torch.allclose(r[0, 0], torch.full((4,), math.log(2.0) + 0.01, dtype=F64))
    assert torch.allclose(q[0, 1], torch.tensor([0.0, 0, 0, 1.0], dtype=F64))
    n, a, b = net.descriptors(q, r)
    assert torch.allclose(n[0, 1], torch.tensor([0.0, 0, 1.0], dtype=F64))
    sp = lambda v: math.log1p(math.exp(v)) + 0.01
    ex, ey = 0.5 * (sp(2.0) + sp(0.0)), 0.5 * (sp(-1.0) + sp(3.0))
    assert math.isclose(float(a[0, 1]), max(ex, ey)) and math.isclose(float(b[0, 1]), min(ex, ey))


def test_quat_to_R_is_rotation():
    rng = np.random.default_rng(1)
    q = torch.tensor(rng.normal(size=(20, 4)), dtype=F64)
    q = q / q.norm(dim=-1, keepdim=True)
    R = net.quat_to_R(q)
    assert torch.allclose(R @ R.transpose(-1, -2), torch.eye(3, dtype=F64).expand(20, 3, 3), atol=1e-12)
    assert torch.allclose(torch.linalg.det(R), torch.ones(20, dtype=F64))
    c, s = math.cos(math.pi / 4), math.sin(math.pi / 4)
    Rz = net.quat_to_R(torch.tensor([c, 0, 0, s], dtype=F64))   # 90 deg about z
    assert torch.allclose(Rz[:, 0], torch.tensor([0.0, 1.0, 0.0], dtype=F64), atol=1e-15)


def test_set_loss_exact_match_and_labels():
    # proposal 1 equals the single target exactly; others far away
    P = 4
    out = torch.zeros(1, P * 12, dtype=F64)
    out[0, 0:3] = torch.tensor([5.0, 5.0, 5.0])
    out[0, 12:15] = torch.tensor([0.1, -0.2, 2.0])
    out[0, 24:27] = torch.tensor([-5.0, 0.0, 1.0])
    out[0, 36:39] = torch.tensor([0.0, 5.0, 1.0])
    c, q, r, s = net.decode(out)
    tgt = (c[0, 1:2].clone(), q[0, 1:2].clone(), r[0, 1:2].clone())
    L = net.set_loss(out, [tgt])
    bce = float(torch.nn.functional.softplus(torch.zeros(P, dtype=F64)).mean()) - 0.0 / P
    # geo term is 0, BCE with y = (0, 1, 0, 0) at logits 0: mean softplus(0) = ln 2
    assert math.isclose(float(L), math.log(2.0), rel_tol=1e-12)
    assert bce == pytest.approx(math.log(2.0))
    # flipping the target normal's sign changes nothing
    qf = net.quat_to_R(tgt[1])
    assert qf.shape == (1, 3, 3)


def test_pair_dist_is_sign_blind_and_zero_on_diagonal():
    rng = np.random.default_rng(2)
    cp = torch.tensor(rng.normal(size=(3, 3)), dtype=F64)
    n = torch.tensor(rng.normal(size=(3, 3)), dtype=F64)
    n = n / n.norm(dim=-1, keepdim=True)
    a = torch.tensor([0.5, 0.3, 0.2], dtype=F64)
    b = torch.tensor([0.1, 0.2, 0.05], dtype=F64)
    D = net.pair_dist(cp, n, a, b, cp, -n, a, b)
    assert torch.allclose(torch.diagonal(D), torch.zeros(3, dtype=F64), atol=1e-15)
    assert torch.allclose(D, D.T, atol=1e-15)


def test_gradient_of_composition_matches_central_differences():
    rng = np.random.default_rng(3)
    prm = net.init_params(seed=4, width=16, n_prop=5)
    for k in prm:
        prm[k] = prm[k].clone().requires_grad_(True)
    X = torch.tensor(rng.normal(size=(2, 11, 3)), dtype=F64)
    tg = []
    for b in range(2):
        ct = torch.tensor(rng.normal(size=(3, 3)), dtype=F64)
        qt = torch.tensor(rng.normal(size=(3, 4)), dtype=F64)
        rt = torch.tensor(rng.uniform(0.1, 0.5, size=(3, 4)), dtype=F64)
        tg.append((ct, qt, rt))

    def f():
        return net.set_loss(net.forward(X, prm, round_bf16=False)["out"], tg)

    L = f()
    L.backward()
    h = 1e-6
    for name in ("W1", "b2", "W3", "Wh", "bh"):
        p = prm[name]
        flat = p.detach().view(-1)
        for idx in rng.choice(flat.numel(), size=4, replace=False):
            old = float(flat[idx])
            with torch.no_grad():
                flat[idx] = old + h
                lp = float(f())
                flat[idx] = old - h
                lm = float(f())
                flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = float(p.grad.view(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)
