"""FP64 CPU oracle for one step of the hybrid nodal-staggered PSATD PIC method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
re-statement of the paper's scheme (Zoni et al., "A hybrid nodal-staggered
pseudo-spectral electromagnetic particle-in-cell method with finite-order
centering", arXiv 2106.12919) in NumPy float64.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library under
``paper_2106_12919_amd/``) never imports, links or calls anything here, and
nothing here imports the product package.

Units are normalised: c = eps0 = mu0 = 1 (the paper is written in SI; setting
the three constants to one keeps every formula visually identical).

Modules
-------
fornberg     Fornberg coefficients and modified wave numbers (Sec. 3, Sec. 4.1)
transforms   the paper's discrete Fourier convention with Yee offsets (App. A)
psatd        standard PSATD coefficients and update on the staggered grid (Sec. 4.2)
centering    finite-order centering nodal <-> staggered (Sec. 3, App. C)
particles    B-spline shapes, nodal gather, relativistic Boris push, deposition
step         one hybrid PIC cycle (Sec. 2, the hybrid cycle)
diagnostics  field energy (Sec. 2 (iii)), relative L2 error (Sec. 5.2), charge; closed-form
             modified wave numbers, centering factor, stencil extent
adjoint      reverse mode of one cycle: conjugate-transposed field solve, transposed
             centering, gather/deposit adjoints, complex-step Boris Jacobians
dft          brute-force DFT used only to pin ``transforms``
"""

from . import fornberg, transforms, psatd, centering, particles, step, diagnostics, adjoint, dft  # noqa: F401
