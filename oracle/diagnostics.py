"""Scalar diagnostics (oracle).

Test infrastructure only (see ``oracle/__init__``).

* field energy W = 1/2 sum_cells (eps0 |E|^2 + |B|^2 / mu0) dV  (Sec. 2, item iii);
* relative L2 error ||F_n - F_h|| / ||F_n||  (Sec. 5.2, eq. ``L2_norm_error``);
* total charge sum_i rho_i dV;
* Gauss residual || [k]_s . E_hat + i rho_hat / eps0 || / || rho_hat / eps0 ||
  (App. A, Gauss's law used in the derivation of the update);
* continuity residual || (rho_hat^{n+1} - rho_hat^n)/dt + i [k]_s . J_hat || / || (rho_hat^{n+1} - rho_hat^n)/dt ||
  (App. A convention; the direct deposition of Sec. 2 does not make it zero);
* stencil extent Gamma of a PSATD coefficient along an axis (Sec. 2 item (ii),
  eq. ``eq_stencil_extent``).
"""

import numpy as np

from . import psatd, transforms
from .transforms import E_NAMES, J_NAMES, OFFSETS

EPS0 = 1.0
MU0 = 1.0


def field_energy(E, B, spacing):
    dV = spacing[0] * spacing[1] * spacing[2]
    e = sum(np.sum(np.asarray(c, dtype=np.float64) ** 2) for c in E)
    b = sum(np.sum(np.asarray(c, dtype=np.float64) ** 2) for c in B)
    return 0.5 * (EPS0 * e + b / MU0) * dV


def rel_l2(ref, test):
    ref = np.asarray(ref, dtype=np.float64)
    test = np.asarray(test, dtype=np.float64)
    den = np.sqrt(np.sum(ref ** 2))
    return float(np.sqrt(np.sum((test - ref) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(test ** 2)))


def total_charge(rho, spacing):
    return float(np.sum(rho) * spacing[0] * spacing[1] * spacing[2])


def gauss_residual(E_stag, rho, spacing, psatd_order, nodal=False):
    """Relative Gauss's-law residual of E on the Yee grid and rho on the nodes, in the paper's
    Fourier convention (App. A).  ``nodal``: every field at the nodes and [k]_c (Sec. 4.1)."""
    shape = rho.shape
    if nodal:
        ks = psatd.centered_wave_vector(shape, spacing, psatd_order)
        Eh = [transforms.forward(E_stag[d], spacing, (0.0, 0.0, 0.0)) for d in range(3)]
    else:
        ks = psatd.staggered_wave_vector(shape, spacing, psatd_order)
        Eh = [transforms.forward(E_stag[d], spacing, OFFSETS[E_NAMES[d]]) for d in range(3)]
    rh = transforms.forward(rho, spacing, OFFSETS["rho"])
    div = ks[0] * Eh[0] + ks[1] * Eh[1] + ks[2] * Eh[2]
    res = div + 1j * rh / EPS0
    den = np.sqrt(np.sum(np.abs(rh / EPS0) ** 2))
    num = np.sqrt(np.sum(np.abs(res) ** 2))
    return float(num / den) if den > 0 else float(num)


def continuity_residual(J, rho_old, rho_new, spacing, dt, psatd_order, nodal=False):
    """Relative continuity residual of J^{n+1/2} (Yee grid; ``nodal``: at the nodes with [k]_c)
    between rho^n and rho^{n+1} on the nodes, in the paper's Fourier convention (App. A)."""
    shape = rho_old.shape
    if nodal:
        ks = psatd.centered_wave_vector(shape, spacing, psatd_order)
        Jh = [transforms.forward(J[d], spacing, (0.0, 0.0, 0.0)) for d in range(3)]
    else:
        ks = psatd.staggered_wave_vector(shape, spacing, psatd_order)
        Jh = [transforms.forward(J[d], spacing, OFFSETS[J_NAMES[d]]) for d in range(3)]
    drho = (transforms.forward(rho_new, spacing, OFFSETS["rho"]) - transforms.forward(rho_old, spacing, OFFSETS["rho"])) / dt
    res = drho + 1j * (ks[0] * Jh[0] + ks[1] * Jh[1] + ks[2] * Jh[2])
    den = np.sqrt(np.sum(np.abs(drho) ** 2))
    num = np.sqrt(np.sum(np.abs(res) ** 2))
    return float(num / den) if den > 0 else float(num)


def stencil_extent(shape, spacing, dt, psatd_order, axis, coefficient, nodal=False):
    """Sec. 2 item (ii), eq. eq_stencil_extent: Gamma(x) = |(1/(N_b N_c)) sum_{k_b,k_c} F^-1_axis[g]|
    for the standard PSATD coefficient ``coefficient`` (one of "C", "S_over_w", "X1", "X2", "X3")
    with [k]_s, or [k]_c for the nodal solver; x = 0 .. n_axis - 1 cells."""
    from . import psatd
    ks = (psatd.centered_wave_vector if nodal else psatd.staggered_wave_vector)(shape, spacing, psatd_order)
    g = np.broadcast_to(psatd.coefficients(ks, dt)[coefficient], shape)
    others = tuple(a for a in range(3) if a != axis)
    return np.abs(np.fft.ifft(g, axis=axis).mean(axis=others))
