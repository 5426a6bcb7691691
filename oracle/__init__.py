"""FP64 CPU oracle for the Wiener reconstruction hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the HIP library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code, tables or helpers with the HIP sources.

Modules (each function cites the passage of the paper it follows):

* ``deposit``     -- fixed-point NGP/CIC/TSC mass assignment onto the (fine)
                     grid (Sec. 3.1.2, def:ngrid).
* ``supersample`` -- ideal low-pass of the 2x deposit and resampling at the
                     target resolution (Sec. 3.1.2), plus a direct-summation
                     evaluator of single cells.
* ``wiener``      -- mean density (eq:nmean), data vector (eq:datamodel with
                     the LSQ noise of eq:noiseav), the Fourier diagonal of
                     S^-1, the operator of eq:WF, and plain conjugate gradients
                     (plus a Fourier-diagonal PCG used only to produce
                     reference solutions faster).

Readings of the paper taken where it is silent are listed in the module
docstrings; every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant or a brute-force evaluation.
"""
from . import deposit, supersample, wiener  # noqa: F401
