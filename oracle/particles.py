"""Macro-particle operations on the nodal grid (oracle).

Test infrastructure only (see ``oracle/__init__``).

The hybrid cycle (Sec. 2) deposits rho and J on the nodal grid and gathers E
and B from the nodal grid; because every nodal component sits at the same
points, one set of shape weights serves all six gathered components (the
momentum-conserving gather, Sec. 2).  The paper names cubic splines as the
shape (Sec. 5.2, 5.3) without printing them.  Reading used: centred
B-splines,
    order 1:  W(d) = 1 - |d|                       (|d| < 1)
    order 3:  W(d) = 2/3 - d^2 + |d|^3/2           (|d| <= 1)
              W(d) = (2 - |d|)^3 / 6               (1 < |d| < 2)
with d the particle-to-node distance in cells; the 3D weight is the product of
the three 1D weights.  The pusher is the relativistic Boris scheme (the paper
itself used the Vay pusher, Sec. 5.2; the relativistic Boris rotation is the
textbook scheme):
    u- = u + (q dt / 2m) E,  gamma- = sqrt(1 + |u-|^2/c^2),
    t = (q dt / (2 m gamma-)) B,  s = 2 t / (1 + |t|^2),
    u' = u- + u- x t,  u+ = u- + u' x s,  u_new = u+ + (q dt / 2m) E.
Positions are absolute float64 coordinates in [0, L) with node i at i*dx.
Deposition (the paper states only the time levels J^{n+1/2}, rho^n, rho^{n+1},
Sec. 4.2): rho^{n+1} from x^{n+1}; J^{n+1/2} = q w v^{n+1/2} S(x^{n+1/2} - x_i)/dV
with x^{n+1/2} = x^n + dt v^{n+1/2} / 2 (direct, not charge-conserving).
"""

import numpy as np

C_LIGHT = 1.0


def shape_1d(order, d):
    """Centred B-spline of the given order (1 or 3) at distance d (cells)."""
    a = np.abs(np.asarray(d, dtype=np.float64))
    if order == 1:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if order == 3:
        inner = 2.0 / 3.0 - a * a + 0.5 * a ** 3
        outer = (2.0 - a) ** 3 / 6.0
        return np.where(a <= 1.0, inner, np.where(a < 2.0, outer, 0.0))
    raise ValueError("shape order must be 1 or 3")


def shape_1d_deriv(order, d):
    """Derivative of ``shape_1d`` with respect to d (taken as 0 at the kinks of order 1)."""
    d = np.asarray(d, dtype=np.float64)
    a = np.abs(d)
    sg = np.sign(d)
    if order == 1:
        return np.where(a < 1.0, -sg, 0.0)
    if order == 3:
        inner = -2.0 * d + 1.5 * d * a
        outer = -0.5 * sg * (2.0 - a) ** 2
        return np.where(a <= 1.0, inner, np.where(a < 2.0, outer, 0.0))
    raise ValueError("shape order must be 1 or 3")


def _axis_nodes(xc, order):
    """[(node index, weight)] along one axis for positions ``xc`` in cells."""
    i0 = np.floor(xc).astype(np.int64)
    offsets = (0, 1) if order == 1 else (-1, 0, 1, 2)
    return [(i0 + o, shape_1d(order, xc - (i0 + o))) for o in offsets]


def _stencil(pos, shape, spacing, order):
    """Yield (linear periodic node index, weight) over the S^3 support nodes."""
    nx, ny, nz = shape
    ax = _axis_nodes(pos[:, 0] / spacing[0], order)
    ay = _axis_nodes(pos[:, 1] / spacing[1], order)
    az = _axis_nodes(pos[:, 2] / spacing[2], order)
    for ix, wx in ax:
        for iy, wy in ay:
            for iz, wz in az:
                lin = (np.mod(ix, nx) * ny + np.mod(iy, ny)) * nz + np.mod(iz, nz)
                yield lin, wx * wy * wz


def gather(fields, pos, spacing, order):
    """Interpolate nodal ``fields`` (list of 3D arrays) to the particle positions: shape (len(fields), Np)."""
    shape = fields[0].shape
    flat = [np.asarray(f, dtype=np.float64).ravel() for f in fields]
    out = np.zeros((len(fields), pos.shape[0]))
    for lin, w in _stencil(pos, shape, spacing, order):
        for c, f in enumerate(flat):
            out[c] += w * f[lin]
    return out


def deposit(values, pos, shape, spacing, order):
    """sum_p values_p S(x_p - x_i) / dV on the nodes, for each array in ``values``."""
    n = int(np.prod(shape))
    dV = spacing[0] * spacing[1] * spacing[2]
    out = [np.zeros(n) for _ in values]
    for lin, w in _stencil(pos, shape, spacing, order):
        for c, v in enumerate(values):
            out[c] += np.bincount(lin, weights=w * v, minlength=n)
    return [o.reshape(shape) / dV for o in out]


def boris(u, E, B, q, m, dt):
    """Relativistic Boris update of u = gamma v (rows x, y, z; shape (3, Np))."""
    k = q * dt / (2.0 * m)
    um = u + k * E
    gm = np.sqrt(1.0 + np.sum(um * um, axis=0) / C_LIGHT ** 2)
    t = (k / gm) * B
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=0))
    up = um + np.cross(um, t, axis=0)
    uplus = um + np.cross(up, s, axis=0)
    return uplus + k * E


def gamma(u):
    return np.sqrt(1.0 + np.sum(u * u, axis=0) / C_LIGHT ** 2)


def wrap(pos, lengths):
    return np.mod(pos, np.asarray(lengths)[None, :])
