"""ps_check_finite counts NaN and infinity exactly (also at the grid-stride
tail and past the 4096-workgroup cap), and the fit loop's opt-in check
refuses to run on non-finite planes (the check runs before any step, so no
kernel sees the planted NaN)."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 255, 257, 4096 * 256 + 77])
def test_check_finite_counts(n):
    from paper_2412_03451_amd.splat import check_finite
    print(f"ps_check_finite n={n}", flush=True)
    rng = np.random.default_rng(n)
    x = rng.normal(size=n).astype(np.float32)
    k = min(n, 37)
    idx = rng.choice(n, size=k, replace=False) if n else np.zeros(0, np.int64)
    vals = np.array([np.nan, np.inf, -np.inf], np.float32)
    x[idx] = vals[np.arange(k) % 3]
    t = torch.as_tensor(x, device="cuda")
    assert check_finite(t) == int((~np.isfinite(x)).sum()) == k
    assert check_finite(torch.ones(5, device="cuda"), t) == k


def test_fit_loop_stops_on_non_finite_planes():
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    from paper_2412_03451_amd.splat import Job, Renderer
    ps = synth.random_planes(32, seed=2)
    cam = synth.tiny_camera()
    r = Renderer([Job(0, ps.K, 0, cam.width, cam.height)], [cam])
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    D, N = r.render(dev(ps.center), dev(ps.quat), dev(ps.radii), torch.tensor([300.0], device="cuda"))
    fit = SceneFit(ps.center, ps.quat, ps.radii, [cam], D.view(1, -1).clone(), N.view(1, -1).clone(),
                   cfg=FitConfig(check_every=4, check_finite=True))
    fit.run(4, graph=False)
    fit.c[3, 1] = float("nan")
    with pytest.raises(FloatingPointError):
        fit.run(4, graph=False)
