"""Plane splitting (oracle).  TEST INFRASTRUCTURE ONLY.

Sec. 3.3 (plane splitting paragraph) and Fig. S1: every 1000 iterations a
plane whose average radii gradient on its X axis (r^{x+}, r^{x-}) exceeds
0.2 is split along its Y axis, and likewise a plane whose average radii
gradient on its Y axis exceeds 0.2 is split along its X axis.  Readings:

* the average radii gradient on the X axis is read as (mean of |dL/dr^{x+}| and of
  |dL/dr^{x-}| over the iterations since the last split in which the plane
  took part in the render, i.e. had a radii gradient that is not all zero)
  averaged over the two: (A[x+] + A[x-]) / (2 n_k) with A the sum of
  magnitudes over those n_k iterations;
* the gradient is that of the per-pixel mean loss (the summed loss of a view
  divided by its pixel count, passed as `scale`).  The threshold 0.2 fixes
  the scale: on the synthetic room most planes cross it at every split under
  the summed loss, and none under the per-pixel mean averaged over all
  iterations instead of the iterations the plane took part in;
* splitting along the Y axis is read as a cut running parallel to the plane's Y axis
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


def split_planes(center, quat, radii, acc, cnt, scale=1.0, thresh: float = 0.2):
    """(center [K',3], quat [K',4], radii [K',4], parent [K']) in float64.
    acc [K,4]: summed |dL/dr|; cnt [K]: iterations with a gradient; scale:
    scalar or [K], from the summed loss to the per-pixel mean."""
    center = np.asarray(center, np.float64)
    quat = np.asarray(quat, np.float64)
    radii = np.asarray(radii, np.float64)
    acc = np.asarray(acc, np.float64)
    import torch
    vx, vy, _ = (t.numpy() for t in quat_to_frame(torch.as_tensor(quat)))
    out_c, out_q, out_r, parent = [], [], [], []
    # the split decision is an integer decided in float32 (the kernels'
    # precision), as average > thresh written without a division:
    # (A+ + A-) scale > thresh (2 n_k)
    f32 = np.float32
    K = center.shape[0]
    cnt = np.asarray(cnt, np.int64).reshape(K)
    scale = np.broadcast_to(np.asarray(scale, np.float64), (K,))
    for k in range(K):
        s = f32(scale[k])
        ct = f32(thresh) * f32(2 * cnt[k])
        # a plane with no iteration counted has no average and is kept
        gx = (f32(acc[k, 0]) + f32(acc[k, 1])) * s if cnt[k] > 0 else f32(0)
        gy = (f32(acc[k, 2]) + f32(acc[k, 3])) * s if cnt[k] > 0 else f32(0)
        rxp, rxm, ryp, rym = radii[k]
        # pieces along X: (offset of the center, radius +, radius -)
        if gx > ct:
            mx, hx = 0.5 * (rxp - rxm), 0.25 * (rxp + rxm)
            xs = [(mx - hx, hx, hx), (mx + hx, hx, hx)]
        else:
            xs = [(0.0, rxp, rxm)]
        if gy > ct:
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
