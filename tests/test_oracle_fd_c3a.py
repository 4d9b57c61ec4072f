"""P7 at the differentiation-check size (CPU only): the oracle's autograd
gradient against the stored float64 central finite differences (h = 1e-6) of
1000 seeded coordinates of 256 rectangles in a 256x192 view, at lambda(0)
and 300 (tests/golden/fd_c3a_*.txt, written by make_fd_c3a.py from the
oracle).  A sample of the stored differences is recomputed here, so the file
cannot drift from the oracle.

Bound: |fd - autograd| <= 5e-5 A + 4 rounding bounds of the difference
+ 1e-9, A the sum over pixels of |per-pixel difference| / 2h.  The 5e-5 is
the truncation of a central difference, h^2 f''' / 6, per pixel: at
lambda = 300 the fringe sigmoid has slope 1500 per metre and its third
derivative reaches ~1e9 per metre cubed, so h = 1e-6 leaves a few 1e-5 of
each pixel's derivative; it is relative to A, not to the sum, where pixel
terms cancel.
"""

import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def load_fd(name):
    rows = np.loadtxt(os.path.join(GOLDEN, f"fd_c3a_{name}.txt"), comments="#")
    coords = [(int(r[0]), int(r[1]), int(r[2])) for r in rows]
    return coords, rows[:, 3], rows[:, 4], rows[:, 5], rows[:, 6].astype(bool)


def fd_scene():
    import sys
    sys.path.insert(0, GOLDEN)
    import make_fd_c3a
    return make_fd_c3a


def fd_bound(absd, err):
    return 5e-5 * absd + 4.0 * err + 1e-9


@pytest.mark.parametrize("name", ["lam0", "lam300"])
def test_autograd_matches_stored_central_differences(name):
    m = fd_scene()
    ps, cam, gD, gN = m.scene()
    lam = m.lambdas()[name]
    coords, fd, err, absd, cont = load_fd(name)
    assert len(coords) == m.N_COORDS and cont.sum() >= 0.8 * len(coords)
    g = oracle.render_backward(ps.center, ps.quat, ps.radii, cam, lam, gD, gN)
    ad = np.array([float(g[w][k, c]) for (w, k, c) in coords])
    dev = np.abs(fd - ad)[cont]
    ratio = dev / fd_bound(absd[cont], err[cont])
    print(f"{name}: {cont.sum()} continuous coordinates, max |fd - autograd| / bound {ratio.max():.3g}, "
          f"max relative {np.max(dev / np.maximum(np.abs(ad[cont]), 1e-12)):.3g}")
    assert np.all(ratio <= 1.0)


@pytest.mark.parametrize("name", ["lam0", "lam300"])
def test_stored_central_differences_are_the_oracles(name):
    """25 of the stored coordinates, recomputed: same continuity decision, same
    difference to within float64 summation order (the host's vector width
    may differ from the machine that wrote the file)."""
    m = fd_scene()
    ps, cam, gD, gN = m.scene()
    lam = m.lambdas()[name]
    coords, fd, err, absd, cont = load_fd(name)
    obj = oracle.fd.FdObjective(ps.center, ps.quat, ps.radii, cam, lam, gD, gN)
    for i in np.linspace(0, len(coords) - 1, 25).round().astype(int):
        f2, e2, _, c2 = obj.central_difference(*coords[i], m.H_STEP)
        assert c2 == cont[i]
        assert abs(f2 - fd[i]) <= 1e-9 * abs(fd[i]) + err[i] + e2
