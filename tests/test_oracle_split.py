"""Pins of the plane-splitting oracle: the children tile the parent's
rectangle exactly (corners in the world frame), thresholds on the average
of the pair of radii gradients, one / two / four children, order."""

import numpy as np

import oracle
from oracle.split import split_planes


def _corners(c, q, r):
    import torch
    vx, vy, _ = (t.numpy() for t in oracle.quat_to_frame(torch.as_tensor(np.asarray(q, np.float64))[None]))
    vx, vy = vx[0], vy[0]
    return {"xmin": -r[1], "xmax": r[0], "ymin": -r[3], "ymax": r[2], "c": np.asarray(c), "vx": vx, "vy": vy}


def _world_box(c, q, r):
    k = _corners(c, q, r)
    return np.array([k["c"] + x * k["vx"] + y * k["vy"] for x in (k["xmin"], k["xmax"]) for y in (k["ymin"], k["ymax"])])


def test_split_x_gives_two_halves_covering_the_parent():
    q = np.array([0.9, 0.1, -0.3, 0.2])
    q /= np.linalg.norm(q)
    c = np.array([1.0, 2.0, 3.0])
    r = np.array([0.5, 0.3, 0.2, 0.4])
    acc = np.array([[3.0, 1.0, 0.0, 0.0]])        # average over x+, x-: (3 + 1) / (2 * 4) = 0.5
    cc, qq, rr, par = split_planes(c[None], q[None], r[None], acc, [4], 1.0, 0.2)
    assert list(par) == [0, 0]
    b0, b1 = _world_box(cc[0], qq[0], rr[0]), _world_box(cc[1], qq[1], rr[1])
    P = _world_box(c, q, r)
    # the two children share the middle edge and together span the parent's corners
    assert np.allclose(rr[0], [0.2, 0.2, 0.2, 0.4]) and np.allclose(rr[1], [0.2, 0.2, 0.2, 0.4])
    assert np.allclose(b0[[0, 1]], P[[0, 1]])        # x = -r^{x-} corners
    assert np.allclose(b1[[2, 3]], P[[2, 3]])        # x = r^{x+} corners
    assert np.allclose(b0[[2, 3]], b1[[0, 1]])       # shared cut
    assert np.allclose(qq, q)


def test_thresholds_and_four_children():
    q = np.array([[1.0, 0, 0, 0]] * 3)
    c = np.zeros((3, 3))
    r = np.array([[0.4, 0.4, 0.2, 0.2]] * 3)
    acc = np.array([[0.19, 0.2, 0.0, 0.0],        # average 0.195 <= 0.2: no split
                    [0.0, 0.0, 0.41, 0.41],       # y only: two children along y
                    [1.0, 1.0, 1.0, 1.0]])        # both: four
    cc, qq, rr, par = split_planes(c, q, r, acc, [1, 1, 1], 1.0, 0.2)
    assert list(par) == [0, 1, 1, 2, 2, 2, 2]
    assert np.allclose(cc[0], 0) and np.allclose(rr[0], r[0])
    assert np.allclose(cc[1], [0, -0.1, 0]) and np.allclose(cc[2], [0, 0.1, 0])
    assert np.allclose(rr[1], [0.4, 0.4, 0.1, 0.1])
    # four children: areas sum to the parent's, centers at the quarter points
    areas = [(x[0] + x[1]) * (x[2] + x[3]) for x in rr[3:]]
    assert np.isclose(sum(areas), (0.8) * (0.4))
    assert np.allclose(sorted(map(tuple, np.round(cc[3:, :2], 12))),
                       sorted([(-0.2, -0.1), (-0.2, 0.1), (0.2, -0.1), (0.2, 0.1)]))


def test_average_over_the_iterations_a_plane_took_part_in():
    """The average divides by each plane's own count and applies its scale;
    a plane that never took part does not split; the comparison is strict."""
    q = np.array([[1.0, 0, 0, 0]] * 5)
    c = np.zeros((5, 3))
    r = np.array([[0.4, 0.4, 0.2, 0.2]] * 5)
    acc = np.array([[30.0, 30.0, 0, 0]] * 5)
    cnt = [100, 200, 0, 100, 150]               # averages 0.3, 0.15, -, 0.3 (scaled 0.03), 0.2 (not > 0.2)
    scale = [1.0, 1.0, 1.0, 0.1, 1.0]
    _, _, _, par = split_planes(c, q, r, acc, cnt, scale, 0.2)
    assert list(par) == [0, 0, 1, 2, 3, 4]
    # the same sums over a per-pixel mean: scale = 1 / pixels of the view
    acc2 = np.array([[0.3 * 2 * 50 * 307200, 0.0, 0, 0]])
    _, _, _, par = split_planes(c[:1], q[:1], r[:1], acc2, [50], 1.0 / 307200, 0.2)
    assert list(par) == [0, 0]
