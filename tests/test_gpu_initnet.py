"""GPU parity of the learned initializer's kernels against the float64
oracle: each point layer from the previous layer's kernel output (bfloat16
activations within one unit in the last place), pooling and head exactly /
to float32 rounding, the set loss and its gradient, the backward's
parameter gradients, and one optimiser step; training on a fixed batch lowers
the loss."""

import numpy as np
import pytest
import torch

import oracle
from oracle import initnet as onet

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _bits_to_f64(t):
    return ((t.to(torch.int32) & 0xFFFF) << 16).view(torch.float32).to(F64).cpu()


def _net(P, seed, head_scale=0.5):
    from paper_2412_03451_amd.initnet import InitNet, he_init, param_views
    flat = he_init(P, seed, head_scale=head_scale)
    net = InitNet(P, params=flat)
    prm = {k: torch.tensor(v.astype(np.float64)) for k, v in param_views(flat, P).items()}
    for k in ("W1", "W2", "W3", "Wh"):
        prm[k] = onet.bf16(prm[k])
    return net, prm


def _points(B, N, seed):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(-2, 2, (B, N)), rng.uniform(-1.5, 1.5, (B, N)), rng.uniform(0.5, 6.0, (B, N))], -1)
    return X.astype(np.float32)


def _ulp_ok(a, b):
    """bfloat16 values equal or one unit in the last place apart; returns the mismatch fraction."""
    d = (a - b).abs()
    bound = torch.maximum(a.abs(), b.abs()) * 2.0 ** -7 + 1e-38
    assert bool((d <= bound).all()), float((d / bound).max())
    return float((d > 0).double().mean())


def test_forward_layers_pool_and_head_match_oracle():
    B, N, P = 2, 512, 16
    net, prm = _net(P, 1)
    X = _points(B, N, 2)
    g, arg, out, dump = net.forward(torch.tensor(X, device="cuda"), dump=True)
    torch.cuda.synchronize()
    h1, h2, h3 = (_bits_to_f64(dump[i]) for i in range(3))
    Xt = torch.tensor(X, dtype=F64).reshape(B * N, 3)
    mism = []
    mism.append(_ulp_ok(h1, onet.bf16(torch.relu(Xt @ prm["W1"] + prm["b1"]))))
    mism.append(_ulp_ok(h2, onet.bf16(torch.relu(h1 @ prm["W2"] + prm["b2"]))))
    mism.append(_ulp_ok(h3, onet.bf16(torch.relu(h2 @ prm["W3"] + prm["b3"]))))
    print("bfloat16 activation mismatch fractions", mism, flush=True)
    assert max(mism) < 0.01
    gref, aref = onet.pool_max(h3.view(B, N, -1))
    assert torch.equal(g.cpu().to(F64), gref)
    assert torch.equal(arg.cpu().to(torch.int64), aref)
    oref = gref @ prm["Wh"] + prm["bh"]
    err = (out.cpu().to(F64) - oref).abs() / (gref.abs() @ prm["Wh"].abs() + prm["bh"].abs() + 1e-30)
    assert float(err.max()) < 1e-5


def _targets(B, seed):
    rng = np.random.default_rng(seed)
    tg, off = [], [0]
    for b in range(B):
        T = int(rng.integers(3, 40)) if b else 1
        c = rng.uniform(-2, 2, (T, 3))
        c[:, 2] += 3.0
        q = rng.normal(size=(T, 4))
        r = rng.uniform(0.05, 0.6, (T, 4))
        tg.append(np.concatenate([c, q, r], 1))
        off.append(off[-1] + T)
    return np.concatenate(tg).astype(np.float32), np.array(off, np.int32)


def test_set_loss_and_gradient_match_oracle():
    from paper_2412_03451_amd.initnet import InitNet
    B, P = 3, 32
    rng = np.random.default_rng(3)
    out = (rng.normal(size=(B, 12 * P)) * 0.5).astype(np.float32)
    out.reshape(B, P, 12)[:, :, 0:3] += np.array([0.0, 0.0, 3.0], np.float32)
    tgt, off = _targets(B, 4)
    net = InitNet(P)
    loss, d_out = net.set_loss(torch.tensor(out, device="cuda"), torch.tensor(tgt, device="cuda"),
                               torch.tensor(off, device="cuda"))
    torch.cuda.synchronize()
    views = [(torch.tensor(tgt[off[b]:off[b + 1], 0:3]), torch.tensor(tgt[off[b]:off[b + 1], 3:7]),
              torch.tensor(tgt[off[b]:off[b + 1], 7:11])) for b in range(B)]
    o64 = torch.tensor(out, dtype=F64, requires_grad=True)
    onet.set_loss(o64, views).backward()
    for b in range(B):
        lb = float(onet.set_loss(torch.tensor(out[b:b + 1], dtype=F64), [views[b]]))
        assert float(loss[b]) == pytest.approx(lb, rel=1e-5)
    ref = o64.grad
    err = (d_out.cpu().to(F64) - ref).abs()
    assert float(err.max()) <= 1e-4 * float(ref.abs().max()) + 1e-7


def _rel(a, b):
    return float((a - b).norm() / max(float(b.norm()), 1e-30))


def test_backward_matches_oracle():
    from paper_2412_03451_amd.initnet import param_views
    B, N, P = 2, 512, 16
    net, prm = _net(P, 5)
    X = _points(B, N, 6)
    Xd = torch.tensor(X, device="cuda")
    g, arg, out = net.forward(Xd)
    rng = np.random.default_rng(7)
    d_out = torch.tensor(rng.normal(size=(B, 12 * P)).astype(np.float32), device="cuda")
    grad = net.backward(Xd, g, arg, d_out)
    torch.cuda.synchronize()
    ref = onet.grads_given_arg(X, prm, arg.cpu(), d_out.cpu())
    got = {k: torch.tensor(v.astype(np.float64)) for k, v in param_views(grad.cpu().numpy(), P).items()}
    # float32 paths (head, layer 3, biases of layers 2 and 3) and bfloat16-operand paths (layers 1 and 2)
    tight = ("Wh", "bh", "W3", "b3", "b2")
    for k in ref:
        r = _rel(got[k], ref[k])
        cs = float((got[k] * ref[k]).sum() / (got[k].norm() * ref[k].norm() + 1e-300))
        print(f"{k}: rel {r:.3g} cosine-1 {cs - 1:.3g}", flush=True)
        assert r <= (1e-4 if k in tight else 2e-2), k
        assert cs >= (1 - 1e-7 if k in tight else 1 - 2e-4), k


def test_adam_and_pack():
    from paper_2412_03451_amd.initnet import InitNet, param_views
    P = 8
    net = InitNet(P, seed=9)
    m0 = net.master.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(8)
    gr = rng.normal(size=m0.size).astype(np.float32)
    net.adam_step(torch.tensor(gr, device="cuda"), lr=1e-3)
    torch.cuda.synchronize()
    ref, _, _ = oracle.adam_step(m0, gr.astype(np.float64), np.zeros_like(m0), np.zeros_like(m0), 1)
    got = net.master.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-6 + 1e-6 * np.abs(ref).max()
    # bfloat16 copies: W2t is W2 transposed, rounded to nearest even
    pv = param_views(got, P)
    C = 256
    w2t = ((net.packed[3 * C:3 * C + C * C].to(torch.int32) & 0xFFFF) << 16).view(torch.float32).cpu()
    assert torch.equal(w2t.view(C, C), onet.bf16(torch.tensor(pv["W2"].T.astype(np.float64))).to(torch.float32))


def test_training_lowers_set_loss():
    from paper_2412_03451_amd.initnet import InitNet
    B, N, P = 4, 256, 32
    X = torch.tensor(_points(B, N, 10), device="cuda")
    tgt, off = _targets(B, 11)
    tgt_d, off_d = torch.tensor(tgt, device="cuda"), torch.tensor(off, device="cuda")
    net = InitNet(P, seed=12)
    first = None
    for it in range(150):
        g, arg, out = net.forward(X)
        loss, d_out = net.set_loss(out, tgt_d, off_d)
        if first is None:
            first = float(loss.mean())
        net.adam_step(net.backward(X, g, arg, d_out), lr=3e-3)
    last = float(loss.mean())
    print(f"set loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.5 * first
