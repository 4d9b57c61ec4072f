"""Shared helpers of the GPU parity tests (inputs and tolerances only)."""

from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24  # float32 unit roundoff


def f32(x) -> float:
    """The float32 value the kernels receive for a scalar input."""
    return float(np.float32(x))


def depth_err(gpu, ref):
    """Error of rendered depth against the float64 reference in units of the
    1e-5 relative bound, |gpu - ref| / (1e-5 * max(|ref|, 1 m)); <= 1 passes."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(gpu - ref) / (1e-5 * np.maximum(np.abs(ref), 1.0))


def normal_err(gpu, ref):
    """Per-component normal error in units of 1e-5 (normals are unit scale)."""
    return np.abs(np.asarray(gpu, np.float64) - np.asarray(ref, np.float64)) / 1e-5


def grad_tol(ref, abssum, rel=1e-4, c=32.0, floor=1e-30):
    """Per-coordinate gradient bound: 1e-4 relative plus c float32 roundoffs of
    the sum over pixels of |contribution| (float32 sums of ~1e4 terms that
    cancel cannot be closer than a few roundoffs of that scale), plus an
    absolute floor for contributions below float32's range."""
    return rel * np.abs(ref) + c * U32 * abssum + floor


def grad_check(gpu, ref, abssum, rel=1e-4, c=32.0, cond=None, c_cond=64.0):
    """(err, tol) per coordinate.  Besides grad_tol, a coordinate is compared
    no finer than 1e-4 of one float32 roundoff of its group's largest
    gradient: below that (hidden planes behind ~30 layers reach 1e-14 of the
    largest gradient) float32 intermediates such as c_j - S_{j+1} of the
    compositing adjoint cannot resolve it.  With cond (the oracle's
    weight_path_magnitude) the bound adds c_cond float32 roundoffs of it:
    dL/dw_j = T_j (c_j - S_{j+1}) cancels inside one pixel when a hit lies
    just in front of a similar one, and its float32 value is off by roundoffs
    of c_j and of S_{j+1}, which sums up to M = 30 hits (64: two roundoffs
    per composited hit, and some)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = grad_tol(ref, np.asarray(abssum, np.float64), rel, c) + rel * U32 * np.abs(ref).max()
    if cond is not None:
        tol = tol + c_cond * U32 * np.asarray(cond, np.float64)
    err = np.abs(gpu - ref)
    return err, tol


def cosine(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
