"""plane_render_fwd_noalloc (the one-job forward whose workspace is the
library's static device array) against the allocating path
(plane_project -> tile_bin -> plane_render_fwd on a caller workspace), called
through the C ABI: the same bits, on two calls in a row, the second with a
smaller input (fewer planes, a smaller image), then a third large call again."""

import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import f32

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _noalloc(lib, ps, cam, lam, tile, prm):
    from paper_2412_03451_amd._lib import check
    from paper_2412_03451_amd.splat import _ptr, _stream, pack_cameras
    c, q, r = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    cams = pack_cameras([cam])
    lt = torch.tensor([lam], device="cuda")
    P = cam.width * cam.height
    depth = torch.full((P,), -7.0, device="cuda")
    normal = torch.full((3 * P,), -7.0, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    pc = prm.c()
    check(lib.plane_render_fwd_noalloc(_ptr(c), _ptr(q), _ptr(r), ps.K, _ptr(cams), cam.width, cam.height,
                                       tile[0], tile[1], _ptr(lt), C.byref(pc), _ptr(depth), _ptr(normal),
                                       _ptr(status), _stream()))
    torch.cuda.synchronize()
    return depth.cpu().numpy(), normal.cpu().numpy(), int(status.item())


def _allocating(ps, cam, lam, tile, prm):
    from paper_2412_03451_amd.splat import Renderer
    r = Renderer.single_scene([cam], ps.K, tile=tile, params=prm)
    D, N = r.render(_dev(ps.center), _dev(ps.quat), _dev(ps.radii), torch.tensor([lam], device="cuda"))
    torch.cuda.synchronize()
    return D.cpu().numpy(), N.cpu().numpy()


def test_noalloc_matches_the_allocating_forward(lib):
    from paper_2412_03451_amd.splat import SplatParams
    gt, info = synth.room_planes(seed=0, target_K=2000)
    init = synth.room_init_planes(gt, seed=1)
    room_cam = synth.room_trajectory(seed=0, n_views=1, info=info)[0]
    tiny = synth.random_planes(64, seed=0)
    tiny_cam = synth.tiny_camera()
    prm = SplatParams()
    calls = [("room 640x480, K=2000, lambda(0)", init, room_cam, f32(oracle.lambda_at(0)), (16, 16)),
             ("tiny 128x96, K=64, lambda 300", tiny, tiny_cam, 300.0, (16, 16)),
             ("room 640x480, K=2000, lambda 300, 8x8 tiles", init, room_cam, 300.0, (8, 8))]
    for name, ps, cam, lam, tile in calls:
        print(f"noalloc call: {name}", flush=True)
        D, N, st = _noalloc(lib, ps, cam, lam, tile, prm)
        Dr, Nr = _allocating(ps, cam, lam, tile, prm)
        assert st == 0
        assert np.array_equal(D.view(np.uint32), Dr.view(np.uint32))
        assert np.array_equal(N.view(np.uint32), Nr.view(np.uint32))
        assert (D > 0).sum() > 0.05 * D.size
