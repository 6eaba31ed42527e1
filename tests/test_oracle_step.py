"""Whole-cycle sanity pins of the oracle (Sec. 2 hybrid cycle).

* a cold plasma with a small sinusoidal velocity perturbation oscillates at the
  plasma frequency w_p = sqrt(n0 q^2 / (eps0 m)) (textbook Langmuir oscillation);
* total charge is conserved exactly by the deposition (partition of unity);
* with the immobile ion background deposited from the initial electrons the
  initial charge density vanishes.
"""

import numpy as np
import pytest

from oracle import diagnostics, particles
from oracle.step import Params, deposit_rho, step


def _cold_plasma(shape, ppc_axis, n0, du, spacing=(1.0, 1.0, 1.0)):
    nx, ny, nz = shape
    g = [(np.arange(n * p) + 0.5) / p for n, p in zip(shape, ppc_axis)]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * np.array(spacing)
    npart = pos.shape[0]
    w = np.full(npart, n0 * np.prod(shape) * np.prod(spacing) / npart)
    k = 2 * np.pi / (nx * spacing[0])
    u = np.zeros((npart, 3))
    u[:, 0] = du * np.sin(k * pos[:, 0])
    return {"pos": pos, "u": u, "w": w, "q": -1.0, "m": 1.0}


def test_langmuir_oscillation_frequency():
    shape, n0, dt = (32, 4, 4), 0.25, 0.5
    wp = np.sqrt(n0)
    p = Params(shape, (1.0, 1.0, 1.0), dt, shape_order=1, center_order=8, psatd_order=16)
    el = _cold_plasma(shape, (2, 1, 1), n0, 1e-3)
    ions = {"pos": el["pos"].copy(), "u": np.zeros_like(el["u"]), "w": el["w"], "q": 1.0, "m": np.inf}
    rho_static = deposit_rho([ions], p)
    zero = [np.zeros(shape) for _ in range(3)]
    state = {"E_stag": [z.copy() for z in zero], "B_stag": [z.copy() for z in zero],
             "rho_old": deposit_rho([el], p, rho_static)}
    assert np.max(np.abs(state["rho_old"])) < 1e-15
    series = []
    nsteps = 60
    for _ in range(nsteps):
        step(state, [el], p, rho_static)
        series.append(state["E_stag"][0][4, 0, 0])
        q = diagnostics.total_charge(state["rho_old"], p.spacing)
        assert abs(q) < 1e-12
    s = np.array(series)
    # zero crossings of E_x at a fixed point: half-period spacing
    t = (np.arange(nsteps) + 1) * dt
    idx = np.where(np.sign(s[:-1]) != np.sign(s[1:]))[0]
    tc = t[idx] - s[idx] * dt / (s[idx + 1] - s[idx])
    half = np.mean(np.diff(tc))
    assert np.pi / half == pytest.approx(wp, rel=0.03)


def test_total_charge_conserved_with_thermal_plasma():
    from paper_2106_12919_amd import inputs
    wl = inputs.small((8, 8, 12), ppc=2, shape_order=3, center_order=4, field_amp=0.01, u_th=0.1)
    p = Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    el = {"pos": wl.electrons.positions(wl.spacing), "u": wl.electrons.u.copy(), "w": wl.electrons.w,
          "q": wl.electrons.q, "m": wl.electrons.m}
    ions = {"pos": wl.ions.positions(wl.spacing), "u": wl.ions.u, "w": wl.ions.w, "q": 1.0, "m": np.inf}
    rho_static = deposit_rho([ions], p)
    state = {"E_stag": wl.E, "B_stag": wl.B, "rho_old": deposit_rho([el], p, rho_static)}
    q0 = np.sum(el["q"] * el["w"])
    for _ in range(3):
        out = step(state, [el], p, rho_static)
        rho_e = out["rho_new"] - rho_static
        assert diagnostics.total_charge(rho_e, p.spacing) == pytest.approx(q0, rel=1e-13)
    assert np.all(particles.gamma(el["u"].T) >= 1.0)


# ---------------------------------------------------------------- fully staggered comparison cycle

def _staggered_params(order):
    from oracle.step import Params
    return Params((10, 12, 10), (1.0, 1.5, 0.75), 0.5, order, 4, 8, staggered=True)


@pytest.mark.parametrize("order", [1, 3])
def test_staggered_gather_reproduces_linear_fields_at_the_particle(order):
    """Each component sampled at its own Yee positions from a linear function is gathered back as
    that function's value at the particle (B-splines reproduce linear functions): the half-cell
    shift per component is right, or the result is off by half a cell times the slope."""
    from oracle import step as ostep
    from oracle.transforms import B_NAMES, E_NAMES, OFFSETS
    p = _staggered_params(order)
    rng = np.random.default_rng(21)
    nx, ny, nz = p.shape
    dx, dy, dz = p.spacing
    g = rng.standard_normal((6, 3)) * 0.01
    fields = []
    for c, name in enumerate(E_NAMES + B_NAMES):
        o = OFFSETS[name]
        X, Y, Z = np.meshgrid((np.arange(nx) + o[0]) * dx, (np.arange(ny) + o[1]) * dy, (np.arange(nz) + o[2]) * dz,
                              indexing="ij")
        fields.append(1.0 + g[c, 0] * X + g[c, 1] * Y + g[c, 2] * Z)
    # particles well inside (the periodic wrap breaks linearity at the edges)
    pos = np.column_stack([rng.uniform(3, nx - 4, 20) * dx, rng.uniform(3, ny - 4, 20) * dy,
                           rng.uniform(3, nz - 4, 20) * dz])
    got = ostep.gather_fields(fields[:3], fields[3:], pos, p)
    for c in range(6):
        np.testing.assert_allclose(got[c], 1.0 + pos @ g[c], atol=1e-13)


@pytest.mark.parametrize("order", [1, 3])
def test_staggered_deposit_is_the_transpose_of_the_staggered_gather(order):
    """<deposit_c(q), F_c> = sum_p q_p gather_c(F_c)(x_p) dV-weighted, component by component, and the
    total of each deposited J component is sum q w v / dV times the cell volume (partition of unity)."""
    from oracle import particles
    from oracle import step as ostep
    p = _staggered_params(order)
    rng = np.random.default_rng(22)
    n = 30
    pos = rng.uniform(0, 1, (n, 3)) * np.asarray(p.lengths)[None, :]
    v = rng.standard_normal((3, n)) * 0.3
    sp = {"q": -1.0, "w": rng.uniform(0.5, 1.5, n)}
    J = ostep.deposit_current(sp, v, pos, p)
    dV = np.prod(p.spacing)
    from oracle.transforms import J_NAMES
    for d in range(3):
        F = rng.standard_normal(p.shape)
        lhs = np.sum(J[d] * F) * dV
        g = particles.gather([F], pos - ostep._yee_shift(J_NAMES[d], p)[None, :], p.spacing, order)[0]
        rhs = np.sum(sp["q"] * sp["w"] * v[d] * g)
        assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + 1)
        assert abs(np.sum(J[d]) * dV - np.sum(sp["q"] * sp["w"] * v[d])) <= 1e-12


# ---------------------------------------------------------------- time level of the deposited current

@pytest.mark.parametrize("axis,sign,v_gal", [(0, 1, 0.0), (1, -1, 0.0), (2, 1, 0.0), (2, 1, -0.3), (0, -1, 0.2)])
def test_current_is_deposited_at_the_half_step_position(axis, sign, v_gal):
    """Sec. 4.2 holds J constant over the step and places it at t^{n+1/2}.  A linear (CIC) weight is
    affine in the particle's coordinate inside a cell, so for a particle that moves along one axis
    without crossing a node, q w v S(x^{n+1/2} - x_i) equals the mean of q w v S(x^n - x_i) and
    q w v S(x^{n+1} - x_i) exactly.  Depositing at x^n or at x^{n+1} (or with a wrong frame shift
    in the Galilean case, where the grid moves with v_gal) breaks the identity by O(v dt)."""
    shape, dt = (8, 6, 10), 0.5
    vg = [0.0, 0.0, 0.0]
    vg[axis] = v_gal
    p = Params(shape, (1.0, 1.0, 1.0), dt, shape_order=1, center_order=4, psatd_order=8, v_gal=tuple(vg))
    rng = np.random.default_rng(31 + axis)
    n = 40
    cells = np.column_stack([rng.integers(0, s, n) for s in shape]).astype(np.float64)
    off = rng.uniform(0.0, 1.0, (n, 3))
    u = np.zeros((n, 3))
    u[:, axis] = sign * rng.uniform(0.2, 0.6, n)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1))
    disp = dt * (u[:, axis] / gam - v_gal)  # motion on the grid along the axis, |disp| < 0.4
    # keep both end points inside the cell along the moving axis
    lo = np.maximum(0.02, -disp + 0.02)
    hi = np.minimum(0.98, 0.98 - disp)
    off[:, axis] = lo + (hi - lo) * rng.uniform(0.0, 1.0, n)
    pos0 = cells + off
    w = rng.uniform(0.5, 1.5, n)
    el = {"pos": pos0.copy(), "u": u.copy(), "w": w, "q": -1.0, "m": 1.0}
    zero = [np.zeros(shape) for _ in range(3)]
    state = {"E_stag": [z.copy() for z in zero], "B_stag": [z.copy() for z in zero],
             "rho_old": deposit_rho([el], p)}
    out = step(state, [el], p)
    pos1 = pos0.copy()
    pos1[:, axis] += disp
    np.testing.assert_allclose(el["pos"], pos1, atol=1e-13)  # E = B = 0: a straight move
    qwv = -1.0 * w * u[:, axis] / gam
    dep = lambda pos: particles.deposit([qwv], pos, shape, p.spacing, 1)[0]
    expect = 0.5 * (dep(pos0) + dep(pos1))
    np.testing.assert_allclose(out["J_nod"][axis], expect, atol=1e-14)
    assert np.max(np.abs(out["J_nod"][axis] - dep(pos1))) > 1e-3  # the end point is measurably different
    for d in range(3):
        if d != axis:
            assert np.max(np.abs(out["J_nod"][d])) == 0.0
