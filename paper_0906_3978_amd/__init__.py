"""MI355X (gfx950) Wiener reconstruction of the galaxy density field.

The HIP library (``libwiener.so``, C ABI in ``include/wiener.h``) grids
galaxies with fixed-point NGP/CIC/TSC assignment and optional 2x
supersampling, and solves the signal-space Wiener filter of Kitaura et al.
(eq:WF, Sec. 3.3.1) by conjugate gradients in FP64 or mixed precision.  This
package is its ctypes binding; see ``Context``.
"""
from ._lib import (Context, Info, Server, WienerError, footprint_bytes, lib, opts,  # noqa: F401
                   SCHEMES, PRECISIONS, STATUS_NAMES, LIB_PATH, SIGNATURES)
