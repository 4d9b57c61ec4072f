"""GPU parity on the method's degenerate cases and at the binning's size limit
(run on an MI355X), against the float64 oracle with the bars of the render
and gradient tests:

* planes that straddle the camera, contain its center, sit inside the near
  distance, lie behind it, are seen nearly edge-on, or sit 5 cm in front of
  it with a fringe covering the whole image (Eq. 4 with the near-distance and
  grazing-ray readings);
* one tile whose list holds 40 (tile, plane) pairs (sorted across the lanes
  of one wave), 200 (one wave, in LDS), 300 and 4096 (one 1024-thread LDS
  sort; 4096 is the longest one such sort takes), 6000 and 20000 (sorted in
  4096-entry chunks, then merged in memory; from 4096 on every pixel
  composites its M = 30 nearest semi-transparent hits); and a list beyond the
  int16 list positions (32767 pairs), which tile_bin must refuse.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import cosine, depth_err, f32, grad_check, normal_err

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _render(ps, cam, lam, tile=(16, 16), capacity=None):
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    r = Renderer.single_scene([cam], ps.K, tile=tile, params=SplatParams(), pair_capacity=capacity)
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], dtype=torch.float32, device="cuda")
    D, N = r.render(c, q, rr, lt)
    torch.cuda.synchronize()
    return r, (c, q, rr, lt), D, N


def _check_forward(r, D, N, ps, cam, lam, label):
    Dg = r.job_depth(D, 0).cpu().numpy()
    Ng = r.job_normal(N, 0).cpu().numpy()
    Dr, Nr, aux = oracle.render(ps.center, ps.quat, ps.radii, cam, f32(lam))
    ed = depth_err(Dg, Dr.numpy())
    en = normal_err(Ng, Nr.numpy())
    print(f"{label}: covered {float((aux['count'] > 0).float().mean()):.3f}, max count {int(aux['count'].max())}, "
          f"max depth err {ed.max():.3g}, max normal err {en.max():.3g} (units of 1e-5)", flush=True)
    assert np.isfinite(Dg).all() and np.isfinite(Ng).all()
    assert ed.max() <= 1.0, np.unravel_index(np.argmax(ed), ed.shape)
    assert en.max() <= 1.0
    return aux


def _check_backward(r, args, ps, cam, lam, seed, label):
    rng = np.random.default_rng(seed)
    gD = rng.normal(size=cam.width * cam.height).astype(np.float32)
    gN = rng.normal(size=(3, cam.width * cam.height)).astype(np.float32)
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, f32(lam), gD, gN)
    # deep stacks of semi-transparent hits: the weight path's cancellation-free
    # magnitude enters the bound as in the full-size tests
    conds = oracle.weight_path_magnitude(ps.center, ps.quat, ps.radii, cam, f32(lam), gD, gN)
    out = r.backward(*args, _dev(gD).reshape(-1), _dev(gN).reshape(-1))
    torch.cuda.synchronize()
    for name, g, gr, s, cd in zip(("center", "quat", "radii"), out, grads, abss, conds):
        g = g.cpu().numpy()
        assert np.isfinite(g).all(), name
        err, tol = grad_check(g, gr.numpy(), s.numpy(), cond=cd.numpy())
        ratio = err / np.maximum(tol, 1e-300)
        cs = cosine(g, gr.numpy())
        print(f"{label} {name}: max err/tol {ratio.max():.3g}, cosine-1 {cs - 1:.3g}", flush=True)
        assert np.all(err <= tol), (name, np.unravel_index(np.argmax(ratio), ratio.shape))
        assert cs >= 1 - 1e-8


@pytest.mark.parametrize("lam", [oracle.lambda_at(0), 300.0])
@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_degenerate_geometry_forward(lam, tile):
    ps = synth.degenerate_planes()
    cam = synth.tiny_camera()
    print(f"degenerate planes K={ps.K} lambda={lam:.4g} tile={tile}", flush=True)
    r, _, D, N = _render(ps, cam, lam, tile)
    _check_forward(r, D, N, ps, cam, lam, f"degenerate lam {lam:.3g} tile {tile}")


@pytest.mark.parametrize("lam", [oracle.lambda_at(0), 60.0])
def test_degenerate_geometry_backward(lam):
    ps = synth.degenerate_planes()
    cam = synth.tiny_camera()
    print(f"degenerate planes backward K={ps.K} lambda={lam:.4g}", flush=True)
    r, args, D, N = _render(ps, cam, lam)
    _check_backward(r, args, ps, cam, lam, seed=5, label=f"degenerate lam {lam:.3g}")
    # the planes never hit get exactly zero gradient
    out = r.backward(*args, _dev(np.ones(cam.width * cam.height, np.float32)),
                     _dev(np.ones(3 * cam.width * cam.height, np.float32)))
    for g in out:
        assert float(g[[1, 4, 5]].abs().max()) == 0.0


@pytest.mark.parametrize("K", [40, 200, 300, 4096, 6000, 20000])
def test_long_tile_lists(K):
    """K planes in one 8x8 tile (30 semi-transparent hits per pixel from 4096
    on, fewer below): up to 64 pairs the list sorts across one wave's lanes, up to 256 in one
    wave's LDS, up to 4096 in one LDS pass of a 1024-thread workgroup, longer
    lists in chunks of 4096 that merge in memory; the sorted list is strictly
    increasing and the maps and gradients match the oracle."""
    K_ = K
    ps = synth.stacked_planes(K_, seed=0)
    cam = synth.tiny_camera(8, 8, 100.0)
    lam = oracle.lambda_at(0)
    print(f"single tile K={K_} lambda={lam:.4g}", flush=True)
    r, args, D, N = _render(ps, cam, lam, (8, 8), capacity=K_ + 64)
    cnt = r.counters()
    assert cnt["pairs"] == K_ and cnt["max_tile"] == K_, cnt
    keys = r.region(10, torch.int64, K_).cpu().numpy().view(np.uint64)
    assert np.all(keys[1:] > keys[:-1])
    assert sorted((keys & np.uint64(0xffffffff)).astype(np.int64).tolist()) == list(range(K_))
    aux = _check_forward(r, D, N, ps, cam, lam, f"single tile {K_}")
    assert int(aux["count"].min()) == 30 if K_ >= 4096 else int(aux["count"].min()) >= 1
    _check_backward(r, args, ps, cam, lam, seed=6, label=f"single tile {K_}")


def test_tile_list_over_the_size_limit_is_refused():
    from paper_2412_03451_amd._lib import PS_ERR_CAPACITY, PlaneSplatError
    K = 32768
    ps = synth.stacked_planes(K, seed=0)
    cam = synth.tiny_camera(8, 8, 100.0)
    print(f"single tile K={K}: expect a capacity error", flush=True)
    with pytest.raises(PlaneSplatError) as e:
        _render(ps, cam, oracle.lambda_at(0), (8, 8), capacity=K + 64)
    assert e.value.code == PS_ERR_CAPACITY
    assert "32767" in str(e.value)


def test_empty_job_in_a_batch_and_empty_scene():
    """A job with an empty plane range renders zeros and leaves the other
    jobs and the gradients bitwise unchanged; a scene without planes (K = 0,
    null plane arrays) renders zeros and differentiates to nothing."""
    from paper_2412_03451_amd.splat import Job, Renderer, adam_step
    ps = synth.random_planes(48, seed=8, independent_radii=True)
    cams = [synth.tiny_camera(), synth.tiny_camera(96, 64, 80.0)]
    K = ps.K
    lam = torch.tensor([20.0], device="cuda")
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    rng = np.random.default_rng(9)
    outs = {}
    for name, jobs in (("with_empty", [Job(0, K, 0, 128, 96), Job(K, K, 1, 96, 64), Job(0, K, 1, 96, 64)]),
                       ("without", [Job(0, K, 0, 128, 96), Job(0, K, 1, 96, 64)])):
        print(f"batch {name}: {len(jobs)} jobs", flush=True)
        r = Renderer(jobs, cams)
        D, N = r.render(c, q, rr, lam)
        P = [j.width * j.height for j in jobs]
        gD = torch.zeros(r.n_pixels, device="cuda")
        gN = torch.zeros(3 * r.n_pixels, device="cuda")
        for s, j in enumerate(jobs):
            if j.plane_end > j.plane_begin:
                o = r.pix_off[s]
                g = torch.as_tensor(np.random.default_rng(100 + j.cam).normal(size=4 * P[s]).astype(np.float32),
                                    device="cuda")
                gD[o:o + P[s]] = g[:P[s]]
                gN[3 * o:3 * (o + P[s])] = g[P[s]:]
        grads = r.backward(c, q, rr, lam, gD, gN)
        torch.cuda.synchronize()
        outs[name] = (r, D, N, [g.clone() for g in grads])
    r1, D1, N1, g1 = outs["with_empty"]
    r0, D0, N0, g0 = outs["without"]
    assert float(r1.job_depth(D1, 1).abs().max()) == 0.0 and float(r1.job_normal(N1, 1).abs().max()) == 0.0
    for s1, s0 in ((0, 0), (2, 1)):
        assert torch.equal(r1.job_depth(D1, s1), r0.job_depth(D0, s0))
        assert torch.equal(r1.job_normal(N1, s1), r0.job_normal(N0, s0))
    for a, b in zip(g1, g0):
        assert torch.equal(a, b)
    # no planes at all
    print("scene without planes", flush=True)
    e = torch.zeros(0, 3, device="cuda"), torch.zeros(0, 4, device="cuda"), torch.zeros(0, 4, device="cuda")
    r = Renderer([Job(0, 0, 0, 128, 96)], cams[:1])
    D, N = r.render(*e, lam)
    assert float(D.abs().max()) == 0.0 and float(N.abs().max()) == 0.0
    gc, gq, gr = r.backward(*e, lam, torch.ones(r.n_pixels, device="cuda"), torch.ones(3 * r.n_pixels, device="cuda"))
    torch.cuda.synchronize()
    assert gc.numel() == gq.numel() == gr.numel() == 0
    m = torch.zeros(0, device="cuda")
    adam_step(*e, gc, gq, gr, m, m.clone(), torch.ones(1, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()


def test_one_launch_step_empty_job_and_empty_scene():
    """plane_render_step with a job without planes in the batch: the other
    jobs' maps, loss and the gradients are those of the batch without it;
    and a scene without planes (K = 0, null plane arrays) renders zeros with
    the loss of empty maps and updates nothing."""
    from paper_2412_03451_amd.splat import Job, Renderer
    ps = synth.random_planes(48, seed=8, independent_radii=True)
    cams = [synth.tiny_camera(), synth.tiny_camera(96, 64, 80.0)]
    K = ps.K
    lam = torch.tensor([20.0], device="cuda")
    tgt = synth.random_planes(48, seed=9, independent_radii=True)
    outs = {}
    for name, jobs in (("with_empty", [Job(0, K, 0, 128, 96), Job(K, K, 1, 96, 64), Job(0, K, 1, 96, 64)]),
                       ("without", [Job(0, K, 0, 128, 96), Job(0, K, 1, 96, 64)])):
        tr = Renderer(jobs, cams)
        tD, tN = tr.render(_dev(tgt.center), _dev(tgt.quat), _dev(tgt.radii), torch.tensor([300.0], device="cuda"))
        r = Renderer(jobs, cams)
        c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
        m, v = torch.zeros(11 * K, device="cuda"), torch.zeros(11 * K, device="cuda")
        loss = torch.empty(len(jobs), 4, device="cuda")
        r.project(c, q, rr, lam)
        r.bin()
        D, N, gD, gN, gc, gq, gr = r.step(tD, tN, m, v, torch.ones(1, dtype=torch.int32, device="cuda"),
                                          loss=loss)
        torch.cuda.synchronize()
        outs[name] = (r, D, N, loss.clone(), [x.clone() for x in (gc, gq, gr, c, q, rr, m, v)])
    r1, D1, N1, l1, g1 = outs["with_empty"]
    r0, D0, N0, l0, g0 = outs["without"]
    assert float(r1.job_depth(D1, 1).abs().max()) == 0.0
    for s1, s0 in ((0, 0), (2, 1)):
        assert torch.equal(r1.job_depth(D1, s1), r0.job_depth(D0, s0))
        assert torch.equal(l1[s1], l0[s0])
    for a, b in zip(g1, g0):
        assert torch.equal(a, b)
    # no planes at all
    e = torch.zeros(0, 3, device="cuda"), torch.zeros(0, 4, device="cuda"), torch.zeros(0, 4, device="cuda")
    r = Renderer([Job(0, 0, 0, 128, 96)], cams[:1])
    tD = torch.ones(r.n_pixels, device="cuda")
    tN = torch.zeros(3 * r.n_pixels, device="cuda")
    r.project(*e, lam)
    r.bin()
    loss = torch.empty(1, 4, device="cuda")
    m0 = torch.zeros(0, device="cuda")
    D, N, gD, gN, gc, gq, gr = r.step(tD, tN, m0, m0.clone(), torch.ones(1, dtype=torch.int32, device="cuda"),
                                      loss=loss)
    torch.cuda.synchronize()
    assert float(D.abs().max()) == 0.0 and float(N.abs().max()) == 0.0
    assert gc.numel() == 0
    # the depth term of empty maps against unit targets: a_d * |0 - 1| per pixel
    assert float(loss[0, 3]) == pytest.approx(r.n_pixels, rel=1e-6)
