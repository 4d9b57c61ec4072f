"""FP64 CPU oracle for planar-primitive splatting (PlanarSplatting, arXiv 2412.03451).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct definition that the GPU kernels are checked against.  Only the test
suite, the package smoke check and the bench's CPU-baseline leg may import it.
It shares no code with the HIP library and imports nothing from it.

Every function brute-forces every pixel against every plane in float64
(torch CPU tensors, so that the gradient is plain reverse-mode autograd of the
forward definition).  Sections cited:

* planar primitive, double radii, local frame ........ Sec. 3.1, Eq. 1-3
* ray-plane intersection ............................. Sec. 3.2, Eq. 4
* in-plane coordinates, rectangle splat weight ....... Sec. 3.2, Eq. 6-9
* lambda schedule .................................... Sec. 3.2, Eq. 10
* filter / per-ray sort / first M / compositing ...... Sec. 3.2, Eq. 11-13
* render loss ........................................ Sec. 3.2, Eq. 14
* Adam, learning rate 1e-3 ........................... Sec. 3.3 and appendix A.2
* plane splitting ..................................... Sec. 3.3, split.py
* initialisation from depth, sphere initialisation ... Sec. 3.1 and 4.3, depth_init.py
* plane merge ........................................ Sec. 3.3, merge.py
* learned initializer (not in the paper; readings) ... initnet.py
* central finite differences of the render .......... fd.py

Readings taken where the paper is silent or garbled are listed in the
docstring of each function.
"""

from .render import (  # noqa: F401
    OracleParams,
    lambda_at,
    quat_to_frame,
    render,
    render_pixels,
    render_tiled,
    order_key,
    footprint_tiles,
)
from .loss import render_loss, loss_terms  # noqa: F401
from .adam import adam_step  # noqa: F401
from .grad import render_backward, per_pixel_abs_grad, weight_path_magnitude  # noqa: F401
from . import initnet  # noqa: F401
from .split import split_planes  # noqa: F401
from . import depth_init  # noqa: F401
from .merge import merge_planes  # noqa: F401
from . import fd  # noqa: F401
