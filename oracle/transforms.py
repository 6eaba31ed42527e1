"""The paper's discrete Fourier convention on the Yee grid (oracle).

Test infrastructure only (see ``oracle/__init__``).

App. A, eqs. ``Fourier_discrete`` and ``Fourier_discrete_staggered``: a
sequence sampled at positions x_j (nodes j*dx or cell centres (j+1/2)*dx) has
the transform  f_hat(k) = sum_j f_j exp(-i k x_j).  In 3D each field component
lives at the Yee position listed at the start of App. A (E^x at (i+1/2, j, k),
..., B^z at (i+1/2, j+1/2, k)); J sits with E and rho is nodal.  With a
component's half-cell offset vector delta this is
    f_hat(k) = exp(-i k . delta) * FFT_index[f](k),
and the inverse is the real part of IFFT_index[exp(+i k . delta) f_hat].
The FFT itself is NumPy's (a library primitive used as one step).
"""

import numpy as np

from .fornberg import k_axis

# Half-cell offsets (in cells) of every component on the Yee grid (App. A list; Sec. 2 schematic).
OFFSETS = {
    "Ex": (0.5, 0.0, 0.0), "Ey": (0.0, 0.5, 0.0), "Ez": (0.0, 0.0, 0.5),
    "Bx": (0.0, 0.5, 0.5), "By": (0.5, 0.0, 0.5), "Bz": (0.5, 0.5, 0.0),
    "Jx": (0.5, 0.0, 0.0), "Jy": (0.0, 0.5, 0.0), "Jz": (0.0, 0.0, 0.5),
    "rho": (0.0, 0.0, 0.0),
}
E_NAMES = ("Ex", "Ey", "Ez")
B_NAMES = ("Bx", "By", "Bz")
J_NAMES = ("Jx", "Jy", "Jz")


def wave_vectors(shape, spacing):
    """Broadcastable 3D arrays (kx, ky, kz) of the grid wave numbers."""
    nx, ny, nz = shape
    dx, dy, dz = spacing
    kx = k_axis(nx, dx)[:, None, None]
    ky = k_axis(ny, dy)[None, :, None]
    kz = k_axis(nz, dz)[None, None, :]
    return kx, ky, kz


def _phase(shape, spacing, offset, sign):
    kx, ky, kz = wave_vectors(shape, spacing)
    dx, dy, dz = spacing
    ox, oy, oz = offset
    return np.exp(sign * 1j * (kx * ox * dx + ky * oy * dy + kz * oz * dz))


def forward(f, spacing, offset):
    """f_hat(k) = sum_j f_j exp(-i k . x_j) with x_j = (j + offset) * spacing."""
    f = np.asarray(f, dtype=np.float64)
    return _phase(f.shape, spacing, offset, -1.0) * np.fft.fftn(f)


def inverse(fh, spacing, offset):
    """Real samples at (j + offset) * spacing from the paper-convention spectrum."""
    return np.fft.ifftn(_phase(fh.shape, spacing, offset, +1.0) * fh).real
