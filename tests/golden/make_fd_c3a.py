"""Writes fd_c3a_lam0.txt and fd_c3a_lam300.txt: float64 central finite
differences (h = 1e-6) of the oracle's render on the differentiation-check
configuration (256 random rectangles, one 256x192 view, f = 200), for 1000
seeded parameter coordinates, at lambda(0) (Eq. 10) and 300.

The objective is sum_p gD_p D_p + gN_p . N_p with seeded upstream gradients
(standard normal, rounded to float32).  Only oracle/ computes the values.
Run from the repository root:  python tests/golden/make_fd_c3a.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

H_STEP = 1e-6
N_COORDS = 1000


def scene():
    ps = synth.random_planes(256, seed=0, independent_radii=True)
    cam = synth.tiny_camera(256, 192, 200.0)
    rng = np.random.default_rng(3)
    P = cam.width * cam.height
    gD = rng.normal(size=P).astype(np.float32)
    gN = rng.normal(size=(3, P)).astype(np.float32)
    return ps, cam, gD, gN


def lambdas():
    return {"lam0": float(np.float32(oracle.lambda_at(0))), "lam300": 300.0}


def main():
    ps, cam, gD, gN = scene()
    coords = oracle.fd.random_coordinates(ps.K, N_COORDS, seed=2)
    for name, lam in lambdas().items():
        t0 = time.time()
        obj = oracle.fd.FdObjective(ps.center, ps.quat, ps.radii, cam, lam, gD, gN)
        lines = [f"# central differences, h = {H_STEP:g}, lambda = {lam!r}; columns: group (0 center, "
                 f"1 quat, 2 radii), plane, component, fd, rounding bound, sum of |pixel differences| / 2h, "
                 f"continuous"]
        for (g, k, c) in coords:
            fd, err, absd, cont = obj.central_difference(g, k, c, H_STEP)
            lines.append(f"{g} {k} {c} {fd!r} {err!r} {absd!r} {int(cont)}")
        with open(os.path.join(HERE, f"fd_c3a_{name}.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
        print(f"{name}: {len(coords)} coordinates in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
