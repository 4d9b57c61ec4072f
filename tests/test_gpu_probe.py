"""The vector-ALU probe used to measure the roofline's issue rate: each lane's
eight chains follow x <- a x + b from x0 = (lane + c) / 1000, whose closed form
after n steps is a^n x0 + b (1 - a^n) / (1 - a)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,rtol", [(0, 1e-5), (1, 1e-12)])
def test_valu_probe_chain_values(kind, rtol):
    from paper_2412_03451_amd.splat import valu_probe
    blocks, iters = 4, 64
    print(f"ps_valu_probe kind={kind} blocks={blocks} iters={iters}", flush=True)
    rate, sink = valu_probe(kind, blocks=blocks, iters=iters, reps=1)
    assert rate > 0
    got = sink.double().cpu().numpy()
    a, b = (np.float32(0.999999), np.float32(1e-6)) if kind == 0 else (0.999999, 1e-6)
    a, b = float(a), float(b)
    lane = np.arange(blocks * 256) % 256
    an = a ** iters
    x0 = (lane[:, None] + np.arange(8)[None, :]) * 1e-3
    want = (an * x0 + b * (1 - an) / (1 - a)).sum(1)
    np.testing.assert_allclose(got, want, rtol=rtol, atol=0)

