"""Adam step on the plane parameters (oracle).  TEST INFRASTRUCTURE ONLY.

The paper optimises centers, radii and rotations with Adam at a fixed
learning rate of 1e-3 (Sec. 3.3, appendix A.2).  It does not state beta or
epsilon; the reading is the usual (0.9, 0.999, 1e-8) with bias correction.
Radii must stay positive (Eq. 1 puts them in R^4_+); after the step they are
clamped to at least r_min.  Quaternions are not renormalised (the renderer
normalises them, Eq. 2-3).
"""

from __future__ import annotations

import numpy as np


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, clamp_min=None):
    """One bias-corrected Adam update in float64.  `step` counts from 1.

    Returns (theta', m', v') as float64 numpy arrays."""
    theta, g, m, v = (np.asarray(x, np.float64) for x in (theta, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    if clamp_min is not None:
        theta = np.maximum(theta, clamp_min)
    return theta, m, v
