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
