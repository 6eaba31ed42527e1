"""Brute-force discrete Fourier transform with explicit sample positions (oracle pin).

Test infrastructure only (see ``oracle/__init__``).

App. A, eqs. ``Fourier_discrete`` / ``Fourier_discrete_staggered`` written out
as the triple sum  f_hat(k) = sum_{i,j,l} f_{ijl} exp(-i k . x_{ijl}),
x_{ijl} = ((i, j, l) + offset) * spacing, for tiny grids only.  It exists to
check ``transforms.forward`` without any FFT.
"""

import numpy as np

from .fornberg import k_axis


def naive_forward(f, spacing, offset):
    f = np.asarray(f, dtype=np.float64)
    nx, ny, nz = f.shape
    kx, ky, kz = k_axis(nx, spacing[0]), k_axis(ny, spacing[1]), k_axis(nz, spacing[2])
    out = np.zeros(f.shape, dtype=np.complex128)
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                acc = 0j
                for i in range(nx):
                    xi = (i + offset[0]) * spacing[0]
                    for j in range(ny):
                        yj = (j + offset[1]) * spacing[1]
                        for l in range(nz):
                            zl = (l + offset[2]) * spacing[2]
                            acc += f[i, j, l] * np.exp(-1j * (kx[a] * xi + ky[b] * yj + kz[c] * zl))
                out[a, b, c] = acc
    return out
