"""Plane splitting (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. 3.3 (plane splitting paragraph) and Fig. S1: every 1000 iterations a
plane whose average radii gradient on its X axis (r^{x+}, r^{x-}) exceeds
0.2 is split along its Y axis, and likewise a plane whose average radii
gradient on its Y axis exceeds 0.2 is split along its X axis.  Readings:

* "average radii gradient on the X axis" = (mean over the iterations since
  the last split of |dL/dr^{x+}| and of |dL/dr^{x-}|) averaged over the two,
  i.e. (A[x+] + A[x-]) / (2 n) with A the sum of magnitudes over n
  iterations; the gradient is that of the loss as this project sums it;
* "split along the Y axis": the cut runs parallel to the plane's Y axis
  through the middle of its X extent, giving two rectangles side by side
  along X, each with half the X extent (both radii along X equal to a
  quarter of the extent, the center moved to the middle of the half), the
  Y radii and the rotation unchanged; a plane over both thresholds is cut
  both ways (four children);
* children of a plane are consecutive and in plane order: [x-, x+] halves,
  each then [y-, y+] halves.
"""

from __future__ import annotations

import numpy as np

from .render import quat_to_frame


def split_planes(center, quat, radii, acc, n_acc: int, thresh: float = 0.2):
    """(center [K',3], quat [K',4], radii [K',4], parent [K']) in float64."""
    center = np.asarray(center, np.float64)
    quat = np.asarray(quat, np.float64)
    radii = np.asarray(radii, np.float64)
    acc = np.asarray(acc, np.float64)
    import torch
    vx, vy, _ = (t.numpy() for t in quat_to_frame(torch.as_tensor(quat)))
    out_c, out_q, out_r, parent = [], [], [], []
    # the split decision is an integer decided in float32 (the kernels' precision)
    f32 = np.float32
    inv = f32(1.0) / (f32(2.0) * f32(n_acc))
    for k in range(center.shape[0]):
        gx = (f32(acc[k, 0]) + f32(acc[k, 1])) * inv
        gy = (f32(acc[k, 2]) + f32(acc[k, 3])) * inv
        rxp, rxm, ryp, rym = radii[k]
        # pieces along X: (offset of the center, radius +, radius -)
        if gx > f32(thresh):
            mx, hx = 0.5 * (rxp - rxm), 0.25 * (rxp + rxm)
            xs = [(mx - hx, hx, hx), (mx + hx, hx, hx)]
        else:
            xs = [(0.0, rxp, rxm)]
        if gy > f32(thresh):
            my, hy = 0.5 * (ryp - rym), 0.25 * (ryp + rym)
            ys = [(my - hy, hy, hy), (my + hy, hy, hy)]
        else:
            ys = [(0.0, ryp, rym)]
        for (ox, xp, xm) in xs:
            for (oy, yp, ym) in ys:
                out_c.append(center[k] + ox * vx[k] + oy * vy[k])
                out_r.append(np.array([xp, xm, yp, ym]))
                out_q.append(quat[k])
                parent.append(k)
    return np.array(out_c), np.array(out_q), np.array(out_r), np.array(parent, np.int64)
