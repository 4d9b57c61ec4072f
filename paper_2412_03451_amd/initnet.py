"""Learned plane initializer: Python front end of the initnet_* kernels.

A point-set network (three point-wise layers of width 256, max over the
points, linear head) maps the back-projected depth samples of a view to P
plane proposals; see include/initnet.h for the definition.  Parameters live
on the device as float32 masters with bfloat16 copies for the MFMA kernels.
"""

from __future__ import annotations


import numpy as np
import torch

from . import _lib
from ._lib import check
from .splat import _ptr, _stream

WIDTH = 256
OUT_PER = 12
TILE = 128


def he_init(P: int, seed: int = 0, head_scale: float = 0.01) -> np.ndarray:
    """Float32 parameter vector (layout of initnet_param_count): He-normal
    point layers, a small head, zero biases."""
    rng = np.random.default_rng(seed)
    C_ = WIDTH
    parts = [
        rng.normal(scale=np.sqrt(2.0 / 3), size=3 * C_), np.zeros(C_),
        rng.normal(scale=np.sqrt(2.0 / C_), size=C_ * C_), np.zeros(C_),
        rng.normal(scale=np.sqrt(2.0 / C_), size=C_ * C_), np.zeros(C_),
        rng.normal(scale=head_scale / np.sqrt(C_), size=C_ * OUT_PER * P), np.zeros(OUT_PER * P),
    ]
    return np.concatenate(parts).astype(np.float32)


def param_views(flat, P: int) -> dict:
    """Named views (W1 [3,C], b1, W2 [C,C], b2, W3, b3, Wh [C,12P], bh) of a flat parameter vector."""
    C_ = WIDTH
    sizes = [("W1", (3, C_)), ("b1", (C_,)), ("W2", (C_, C_)), ("b2", (C_,)), ("W3", (C_, C_)), ("b3", (C_,)),
             ("Wh", (C_, OUT_PER * P)), ("bh", (OUT_PER * P,))]
    out, o = {}, 0
    for name, shp in sizes:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


class InitNet:
    def __init__(self, P: int = 256, seed: int = 0, device="cuda", params: np.ndarray | None = None):
        self.lib = _lib.load()
        self.P = P
        self.device = torch.device(device)
        n = int(self.lib.initnet_param_count(P))
        if n <= 0:
            raise ValueError(f"InitNet: bad proposal count {P}")
        init = he_init(P, seed) if params is None else np.asarray(params, np.float32)
        assert init.size == n
        self.master = torch.tensor(init, device=self.device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.step_no = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.packed = torch.empty(int(self.lib.initnet_packed_count(P)), dtype=torch.int16, device=self.device)
        self.pack()

    def pack(self):
        check(self.lib.initnet_pack(_ptr(self.master), self.P, _ptr(self.packed), _stream()))

    def forward(self, X: torch.Tensor, dump: bool = False):
        """X [B, N, 3] float32 (N a multiple of 128) -> g [B, C], arg [B, C], out [B, 12P]
        (and the h1, h2, h3 activations [3, B*N, C] as bfloat16 bits if dump)."""
        X = X.contiguous()
        B, N = int(X.shape[0]), int(X.shape[1])
        ws = torch.empty(int(self.lib.initnet_forward_ws(B, N)), dtype=torch.float32, device=self.device)
        if ws.numel() == 0:
            raise ValueError(f"InitNet.forward: N={N} must be a positive multiple of {TILE}")
        g = torch.empty(B, WIDTH, dtype=torch.float32, device=self.device)
        arg = torch.empty(B, WIDTH, dtype=torch.int32, device=self.device)
        out = torch.empty(B, OUT_PER * self.P, dtype=torch.float32, device=self.device)
        dmp = torch.empty(3, B * N, WIDTH, dtype=torch.int16, device=self.device) if dump else None
        check(self.lib.initnet_forward(_ptr(self.master), _ptr(self.packed), self.P, _ptr(X), B, N, _ptr(g),
                                       _ptr(arg), _ptr(out), _ptr(ws), _ptr(dmp), _stream()))
        return (g, arg, out, dmp) if dump else (g, arg, out)

    def set_loss(self, out: torch.Tensor, tgt: torch.Tensor, tgt_off: torch.Tensor):
        """Set loss per view [B] and d(mean loss)/d out [B, 12P]; tgt [T, 11]
        (center, quaternion, radii), tgt_off [B+1] int32 row offsets."""
        B = int(out.shape[0])
        loss = torch.empty(B, dtype=torch.float32, device=self.device)
        d_out = torch.empty_like(out)
        check(self.lib.initnet_set_loss(_ptr(out.contiguous()), B, self.P, _ptr(tgt.contiguous()),
                                        _ptr(tgt_off.contiguous()), _ptr(loss), _ptr(d_out), _stream()))
        return loss, d_out

    def backward(self, X, g, arg, d_out) -> torch.Tensor:
        """Gradient of sum(d_out * out) with respect to the float32 parameters."""
        B, N = int(X.shape[0]), int(X.shape[1])
        n = int(self.lib.initnet_backward_ws(B, self.P))
        if n <= 0:
            raise ValueError(f"InitNet.backward: B={B} must be even")
        ws = torch.empty(n, dtype=torch.float32, device=self.device)
        grad = torch.empty_like(self.master)
        check(self.lib.initnet_backward(_ptr(self.master), _ptr(self.packed), self.P, _ptr(X.contiguous()), B, N,
                                        _ptr(g), _ptr(arg), _ptr(d_out.contiguous()), _ptr(grad), _ptr(ws),
                                        _stream()))
        return grad

    def adam_step(self, grad, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        self.step_no += 1
        check(self.lib.initnet_adam(_ptr(self.master), _ptr(self.m), _ptr(self.v), _ptr(grad), self.master.numel(),
                                    _ptr(self.step_no), lr, betas[0], betas[1], eps, _stream()))
        self.pack()
