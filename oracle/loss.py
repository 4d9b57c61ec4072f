"""Render loss of Eq. 14 (oracle).  TEST INFRASTRUCTURE ONLY.

Reading of Eq. 14 (its parentheses are garbled in print):

    L = a_cos * sum_r |1 - N(r) . N_pre(r)|
      + a_nl1 * sum_r ||N(r) - N_pre(r)||_1
      + a_d   * sum_r |D(r) - D_pre(r)|

with a_cos = a_nl1 = alpha_1 = 5 and a_d = alpha_2 = 1, summed over the
pixels (reduction "sum", as printed; "mean" divides each sum by the number
of pixels counted).  An optional mask drops pixels.  Images are laid out as
depth [..., H, W] and normal [..., 3, H, W]; the component axis is -3.
"""

from __future__ import annotations

import torch

F64 = torch.float64


def loss_terms(D, N, Dt, Nt, mask=None, a_cos=5.0, a_nl1=5.0, a_d=1.0, reduction="sum"):
    """The three weighted sums of Eq. 14 as float64 scalars (differentiable)."""
    D, N, Dt, Nt = (torch.as_tensor(x).to(F64) for x in (D, N, Dt, Nt))
    cos_t = (1 - (N * Nt).sum(-3)).abs()
    nl1_t = (N - Nt).abs().sum(-3)
    d_t = (D - Dt).abs()
    if mask is not None:
        m = torch.as_tensor(mask).to(F64)
        cos_t, nl1_t, d_t = cos_t * m, nl1_t * m, d_t * m
        cnt = m.sum()
    else:
        cnt = torch.tensor(float(D.numel()), dtype=F64)
    terms = [a_cos * cos_t.sum(), a_nl1 * nl1_t.sum(), a_d * d_t.sum()]
    if reduction == "mean":
        terms = [x / cnt for x in terms]
    return terms


def render_loss(D, N, Dt, Nt, **kw):
    """Total loss (sum of the three terms)."""
    a, b, c = loss_terms(D, N, Dt, Nt, **kw)
    return a + b + c
