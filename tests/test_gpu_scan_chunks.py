"""Binning of a batch larger than one scan chunk (4096 tiles and 4096
records per scan workgroup): 14 jobs of 640x480 in 8x8 tiles (67 200 tiles)
over 700 planes each (9 800 records) render, in one batched call, the bits
that each job gives rendered alone (one chunk), and the backward gives the
gradients of the separate calls summed in job order to within float32
roundoff of the sum.  Exercises the chunk bases of the tile and record
offsets and the last-workgroup combination of the scan."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def test_multi_chunk_batch_equals_separate_renders():
    from paper_2412_03451_amd.splat import Job, Renderer
    gt, info = synth.room_planes(seed=21, target_K=700)
    cams = synth.room_trajectory(21, 14, info, width=640, height=480, f=577.0)
    K = gt.K
    c, q, r = _dev(gt.center), _dev(gt.quat), _dev(gt.radii)
    lam = torch.tensor([40.0], device="cuda")
    jobs = [Job(0, K, v, 640, 480, (8, 8)) for v in range(len(cams))]
    big = Renderer(jobs, cams, pair_capacity=1 << 22)
    print(f"tiles {big.L.n_tiles}, records {big.L.n_records}, items {big.L.n_items}", flush=True)
    assert big.L.n_tiles > 2 * 4096 and big.L.n_records > 2 * 4096
    D, N = big.render(c, q, r, lam)
    rng = np.random.default_rng(5)
    gD = _dev(rng.normal(size=D.shape[0]))
    gN = _dev(rng.normal(size=N.shape[0]))
    gc, gq, gr = big.backward(c, q, r, lam, gD, gN)
    torch.cuda.synchronize()
    HW = 640 * 480
    acc = [np.zeros((K, 3)), np.zeros((K, 4)), np.zeros((K, 4))]
    mag = [np.zeros((K, 3)), np.zeros((K, 4)), np.zeros((K, 4))]
    for v in range(len(cams)):
        one = Renderer([Job(0, K, v, 640, 480, (8, 8))], cams, pair_capacity=1 << 20)
        d1, n1 = one.render(c, q, r, lam)
        assert torch.equal(d1, D[v * HW:(v + 1) * HW]), v
        assert torch.equal(n1, N[3 * v * HW:3 * (v + 1) * HW]), v
        g1 = one.backward(c, q, r, lam, gD[v * HW:(v + 1) * HW].contiguous(),
                          gN[3 * v * HW:3 * (v + 1) * HW].contiguous())
        for i in range(3):
            x = g1[i].double().cpu().numpy()
            acc[i] += x
            mag[i] += np.abs(x)
    for i, g in enumerate((gc, gq, gr)):
        got = g.double().cpu().numpy()
        bound = 64 * np.float32(2 ** -24) * mag[i] + 1e-30
        assert np.all(np.abs(got - acc[i]) <= bound), i
