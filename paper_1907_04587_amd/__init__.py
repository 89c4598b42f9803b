"""MI355X non-smooth Newton solver for rigid, articulated and tetrahedral-FEM bodies
with contact and smooth isotropic friction (Macklin et al., TOG 2019).

The solver runs in libnsn.so (hand-written HIP kernels for gfx950, C ABI in
include/nsn.h).  This package only marshals arguments: torch provides the device
workspace and the stream.
"""
from .scene import Scene, params_c, stats_to_dicts  # noqa: F401
from ._lib import NSNError, lib  # noqa: F401
