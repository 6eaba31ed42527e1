"""Seeded synthetic inputs for the hybrid PSATD PIC step.

This module only draws random numbers and samples initial conditions; it holds
none of the method's arithmetic (no Fornberg coefficients, no modified wave
numbers, no PSATD coefficients, no shape functions).  Both the HIP path and the
CPU oracle receive its outputs.

Every workload is normalised (c = eps0 = mu0 = 1, electron charge -1, mass 1,
cell size 1, c*dt = 0.5 cells).  Particles are generated cell-major: for every
cell of the plasma region, ``ppc`` particles with float64 offsets drawn
uniformly in [0, 1)^3, then momenta u = gamma*v drawn per component from
N(0, u_th^2).  The generator is NumPy's PCG64 seeded per workload.
Immobile neutralising ions sit on the initial electron positions; each side
deposits them once into the static charge background.

The beam-driven configuration adds a cold electron beam (Gaussian density, 8 particles per cell
inside 3 sigma, weights from the density at each particle) to a 1-ppc cold plasma, and starts
from the beam's relativistic self-fields, solved from its continuous density with the exact wave
vector and sampled at the Yee positions; only the plasma is neutralised by ions.

The laser of the two laser configurations is sampled at each component's Yee
position, E_x = E0 exp(-r^2/w0^2) exp(-(z-z0)^2/L^2) cos(k0 (z-z0)), B_y = E_x,
with E0 = a0 * omega0, k0 = omega0 = 2 pi / wavelength, L = FWHM / (2 sqrt(ln 2)),
and then made divergence-free by removing the longitudinal part with the exact
(continuum) wave vector, so that the initial state satisfies Gauss's law with
zero net charge.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Yee offsets (cells) of the staggered components, used only to sample the laser.
_YEE = {
    "Ex": (0.5, 0.0, 0.0), "Ey": (0.0, 0.5, 0.0), "Ez": (0.0, 0.0, 0.5),
    "Bx": (0.0, 0.5, 0.5), "By": (0.5, 0.0, 0.5), "Bz": (0.5, 0.5, 0.0),
}


@dataclass
class Species:
    cell: np.ndarray        # (Np, 3) int64 cell indices (i, j, k)
    off: np.ndarray         # (Np, 3) float64 offsets in [0, 1)
    u: np.ndarray           # (Np, 3) float64 momenta gamma*v/c
    w: np.ndarray           # (Np,) float64 macro weights
    q: float = -1.0
    m: float = 1.0

    @property
    def n(self):
        return int(self.cell.shape[0])

    def positions(self, spacing):
        """Absolute positions (Np, 3) in float64."""
        return (self.cell + self.off) * np.asarray(spacing, dtype=np.float64)[None, :]


@dataclass
class Workload:
    name: str
    shape: tuple
    spacing: tuple
    dt: float
    shape_order: int
    center_order: int
    psatd_order: int
    dtype: str                       # "f32" or "f64"
    steps: int
    electrons: Species
    ions: Optional[Species]          # immobile background (deposited once, rho_static)
    E: list = field(default_factory=list)   # 3 arrays on the Yee grid
    B: list = field(default_factory=list)

    @property
    def cells(self):
        return int(np.prod(self.shape))


def uniform_plasma(rng, shape, ppc, n0, u_th, z_min=0):
    """Cell-major uniform plasma in the cells with k >= z_min."""
    nx, ny, nz = shape
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(z_min, nz), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.int64)
    cell = np.repeat(cells, ppc, axis=0)
    n = cell.shape[0]
    off = rng.random((n, 3))
    u = rng.normal(0.0, u_th, (n, 3)) if u_th > 0 else np.zeros((n, 3))
    w = np.full(n, n0 / ppc)
    return Species(cell=cell, off=off, u=u, w=w, q=-1.0, m=1.0)


def ions_of(electrons):
    return Species(cell=electrons.cell, off=electrons.off, u=np.zeros_like(electrons.u),
                   w=electrons.w, q=+1.0, m=np.inf)


def _divergence_free(comps, names, spacing):
    """Remove the longitudinal part of a sampled vector field with the exact wave vector."""
    shape = comps[0].shape
    ks = [2 * np.pi * np.fft.fftfreq(n, d) for n, d in zip(shape, spacing)]
    K = np.meshgrid(*ks, indexing="ij")
    ph = []
    for name in names:
        o = _YEE[name]
        ph.append(np.exp(-1j * (K[0] * o[0] * spacing[0] + K[1] * o[1] * spacing[1] + K[2] * o[2] * spacing[2])))
    F = [ph[c] * np.fft.fftn(comps[c]) for c in range(3)]
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    k2[0, 0, 0] = 1.0
    kdotF = (K[0] * F[0] + K[1] * F[1] + K[2] * F[2]) / k2
    F = [F[c] - K[c] * kdotF for c in range(3)]
    return [np.fft.ifftn(F[c] / ph[c]).real for c in range(3)]


def laser_fields(shape, spacing, a0, wavelength, waist, fwhm, z0):
    """Divergence-free Gaussian laser polarised along x, propagating along +z."""
    nx, ny, nz = shape
    k0 = 2 * np.pi / wavelength
    E0 = a0 * k0
    L = fwhm / (2 * np.sqrt(np.log(2.0)))
    xc, yc = 0.5 * nx * spacing[0], 0.5 * ny * spacing[1]

    def sample(name):
        o = _YEE[name]
        x = (np.arange(nx) + o[0]) * spacing[0]
        y = (np.arange(ny) + o[1]) * spacing[1]
        z = (np.arange(nz) + o[2]) * spacing[2]
        X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
        r2 = (X - xc) ** 2 + (Y - yc) ** 2
        return E0 * np.exp(-r2 / waist ** 2) * np.exp(-((Z - z0) ** 2) / L ** 2) * np.cos(k0 * (Z - z0))

    zero = np.zeros(shape)
    E = _divergence_free([sample("Ex"), zero, zero], ("Ex", "Ey", "Ez"), spacing)
    B = _divergence_free([zero, sample("By"), zero], ("Bx", "By", "Bz"), spacing)
    return E, B


def beam_plasma(rng, shape, n0, gamma, sigma_r, sigma_z, center, ppc_beam=8, extent=3.0):
    """Cold plasma at 1 particle per cell everywhere plus a cold electron drive beam: 8 particles
    per cell in the cells whose centres lie inside the ellipsoid of semi-axes 3 sigma, moving
    along +z with Lorentz factor gamma, weights n_b(x_p) dV / ppc_beam with the Gaussian density
    n_b = n0 exp(-r^2 / (2 sigma_r^2) - (z - z_c)^2 / (2 sigma_z^2)) (peak n0)."""
    plasma = uniform_plasma(rng, shape, 1, n0, 0.0)
    xc, yc, zc = center
    r = [np.arange(int(np.floor(c - extent * s)), int(np.ceil(c + extent * s)) + 1)
         for c, s in ((xc, sigma_r), (yc, sigma_r), (zc, sigma_z))]
    ii, jj, kk = np.meshgrid(*r, indexing="ij")
    inside = (((ii + 0.5 - xc) / (extent * sigma_r)) ** 2 + ((jj + 0.5 - yc) / (extent * sigma_r)) ** 2
              + ((kk + 0.5 - zc) / (extent * sigma_z)) ** 2) <= 1.0
    cells = np.stack([ii[inside], jj[inside], kk[inside]], axis=1).astype(np.int64)
    cell = np.repeat(cells, ppc_beam, axis=0)
    n = cell.shape[0]
    off = rng.random((n, 3))
    pos = cell + off
    nb = n0 * np.exp(-((pos[:, 0] - xc) ** 2 + (pos[:, 1] - yc) ** 2) / (2 * sigma_r ** 2)
                     - (pos[:, 2] - zc) ** 2 / (2 * sigma_z ** 2))
    u = np.zeros((n, 3))
    u[:, 2] = np.sqrt(gamma ** 2 - 1.0)
    beam = Species(cell=cell % np.asarray(shape)[None, :], off=off, u=u, w=nb / ppc_beam, q=-1.0, m=1.0)
    electrons = Species(cell=np.concatenate([plasma.cell, beam.cell]), off=np.concatenate([plasma.off, beam.off]),
                        u=np.concatenate([plasma.u, beam.u]), w=np.concatenate([plasma.w, beam.w]))
    return electrons, plasma


def beam_fields(shape, spacing, n0, gamma, sigma_r, sigma_z, center):
    """Self-fields of the beam's (continuous) Gaussian charge density -n_b, moving along +z at
    beta = sqrt(1 - 1/gamma^2): phi = rho / (kx^2 + ky^2 + kz^2 / gamma^2),
    E = -i (kx, ky, kz / gamma^2) phi, B = beta z x E, with the exact (continuum) wave vector,
    k = 0 set to zero, each component sampled at its Yee position (FFTs of scipy, threaded)."""
    import scipy.fft as sfft
    nx, ny, nz = shape
    xc, yc, zc = center
    X = (np.arange(nx) - xc)[:, None, None]
    Y = (np.arange(ny) - yc)[None, :, None]
    Z = (np.arange(nz) - zc)[None, None, :]
    rho = -(n0 * np.exp(-(X * X) / (2 * sigma_r ** 2)) * np.exp(-(Y * Y) / (2 * sigma_r ** 2))
            * np.exp(-(Z * Z) / (2 * sigma_z ** 2)))
    rh = sfft.fftn(rho.astype(np.complex128), workers=-1)
    del rho
    kx = (2 * np.pi * np.fft.fftfreq(nx, spacing[0]))[:, None, None]
    ky = (2 * np.pi * np.fft.fftfreq(ny, spacing[1]))[None, :, None]
    kz = (2 * np.pi * np.fft.fftfreq(nz, spacing[2]))[None, None, :]
    den = kx * kx + ky * ky + kz * kz / gamma ** 2
    den[0, 0, 0] = 1.0
    rh /= den
    rh[0, 0, 0] = 0.0
    del den
    beta = np.sqrt(1.0 - 1.0 / gamma ** 2)

    def at(name, comp):  # real samples at the component's Yee positions of the spectrum comp
        o = _YEE[name]
        ph = (np.exp(1j * kx * o[0] * spacing[0]) * np.exp(1j * ky * o[1] * spacing[1])
              * np.exp(1j * kz * o[2] * spacing[2]))
        return sfft.ifftn(comp * ph, workers=-1).real

    Ex = at("Ex", -1j * kx * rh)
    Ey = at("Ey", -1j * ky * rh)
    Ez = at("Ez", -1j * kz / gamma ** 2 * rh)
    # B = beta z x E: (Bx, By, Bz) = (-beta Ey, beta Ex, 0), at the B components' own positions
    Bx = at("Bx", 1j * beta * ky * rh)
    By = at("By", -1j * beta * kx * rh)
    return [Ex, Ey, Ez], [Bx, By, np.zeros(shape)]


def config(name, dtype=None, center_order=None, seed=None):
    """The named workloads (see the module docstring for the common recipe)."""
    if name == "thermal32":
        # 32^3 periodic thermal plasma, 8 ppc, u_th = 0.01, CIC, centering order 8, float64, 10 steps.
        shape, ppc, u_th, n0 = (32, 32, 32), 8, 0.01, 0.01
        rng = np.random.Generator(np.random.PCG64(1001 if seed is None else seed))
        el = uniform_plasma(rng, shape, ppc, n0, u_th)
        zero = [np.zeros(shape) for _ in range(3)]
        return Workload(name, shape, (1.0, 1.0, 1.0), 0.5, 1, center_order or 8, 16, dtype or "f64", 10,
                        el, ions_of(el), [z.copy() for z in zero], [z.copy() for z in zero])
    if name in ("laser128", "laser64"):
        if name == "laser128":
            # 128x128x256, laser a0=2, lambda=16, waist 20, FWHM 30, into 2 ppc cold plasma for z >= 64;
            # cubic shape, centering order 16, float32, 200 steps.
            shape, ppc, zmin, a0, waist, corder, steps, sd = (128, 128, 256), 2, 64, 2.0, 20.0, 16, 200, 1002
        else:
            # 64x64x128, laser a0=1, lambda=16, waist 12, FWHM 30, 4 ppc cold plasma everywhere;
            # cubic shape, centering order 8, float32, 60 steps.
            shape, ppc, zmin, a0, waist, corder, steps, sd = (64, 64, 128), 4, 0, 1.0, 12.0, 8, 60, 1004
        omega0 = 2 * np.pi / 16.0
        n0 = 0.01 * omega0 ** 2
        rng = np.random.Generator(np.random.PCG64(sd if seed is None else seed))
        el = uniform_plasma(rng, shape, ppc, n0, 0.0, z_min=zmin)
        E, B = laser_fields(shape, (1.0, 1.0, 1.0), a0, 16.0, waist, 30.0, 32.0)
        return Workload(name, shape, (1.0, 1.0, 1.0), 0.5, 3, center_order or corder, 16, dtype or "f32",
                        steps, el, ions_of(el), E, B)
    if name in ("beam384", "beam96"):
        # Beam-driven wake: 384x384x768 (beam96: the same setup scaled by 1/4 per axis, for tests),
        # plasma 1 ppc cold everywhere at n0 = 2/256 (k_p sigma_z = sqrt 2 with sigma_z = 16), electron
        # drive beam sigma_r = 8, sigma_z = 16, gamma = 1000, 8 ppc inside 3 sigma, centred at
        # (192, 192, 576) (scaled); cubic shape, centering order 16, float32, 100 steps.
        sc = 1 if name == "beam384" else 4
        shape = (384 // sc, 384 // sc, 768 // sc)
        n0, gamma, sr, sz = 2.0 / 256.0, 1000.0, 8.0 / sc, 16.0 / sc
        center = (192.0 / sc, 192.0 / sc, 576.0 / sc)
        rng = np.random.Generator(np.random.PCG64(1005 if seed is None else seed))
        el, plasma = beam_plasma(rng, shape, n0, gamma, sr, sz, center)
        E, B = beam_fields(shape, (1.0, 1.0, 1.0), n0, gamma, sr, sz, center)
        return Workload(name, shape, (1.0, 1.0, 1.0), 0.5, 3, center_order or 16, 16, dtype or "f32", 100,
                        el, ions_of(plasma), E, B)
    if name == "thermal256":
        # 256^3 periodic thermal plasma, 8 ppc, u_th = 0.05, CIC, centering order swept, 20 steps.
        shape, ppc, u_th, n0 = (256, 256, 256), 8, 0.05, 0.01
        rng = np.random.Generator(np.random.PCG64(1003 if seed is None else seed))
        el = uniform_plasma(rng, shape, ppc, n0, u_th)
        zero = [np.zeros(shape) for _ in range(3)]
        return Workload(name, shape, (1.0, 1.0, 1.0), 0.5, 1, center_order or 8, 16, dtype or "f32", 20,
                        el, ions_of(el), [z.copy() for z in zero], [z.copy() for z in zero])
    raise KeyError(name)


def small(shape, ppc=2, shape_order=1, center_order=4, psatd_order=16, dtype="f64", u_th=0.05,
          field_amp=0.05, seed=7, dt=0.5, spacing=(1.0, 1.0, 1.0), with_ions=True):
    """A small random workload for parity tests: thermal plasma plus random fields on every component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    el = uniform_plasma(rng, shape, ppc, 0.01, u_th)
    E = [field_amp * rng.standard_normal(shape) for _ in range(3)]
    B = [field_amp * rng.standard_normal(shape) for _ in range(3)]
    return Workload("small", tuple(shape), tuple(spacing), dt, shape_order, center_order, psatd_order, dtype, 1,
                    el, ions_of(el) if with_ions else None, E, B)


def random_grid(shape, seed, count=1, amp=1.0):
    """``count`` standard-normal float64 arrays of ``shape`` (for kernel-level tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [amp * rng.standard_normal(shape) for _ in range(count)]
