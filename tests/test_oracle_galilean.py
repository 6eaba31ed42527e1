"""Pins of the oracle's standard Galilean PSATD (Sec. 4.3): the v_gal -> 0 limit is the standard
update (Sec. 4.3 remark), the vacuum update's eigenvalues give the dispersion relation of App. B,
and the update integrates the Galilean Fourier-space Maxwell equations exactly over a step
(checked against a high-accuracy numerical ODE integration) with sources obeying the Galilean
continuity equation, preserving Gauss's law.  CPU only."""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import psatd
from oracle.fornberg import k_axis, k_centered, k_staggered


def _grid_k(shape, order):
    ks = psatd.staggered_wave_vector(shape, (1.0, 1.0, 1.0), order)
    kc = psatd.centered_wave_vector(shape, (1.0, 1.0, 1.0), order)
    return ks, kc


def test_small_galilean_velocity_approaches_standard():
    shape, dt = (8, 12, 16), 0.5
    ks, kc = _grid_k(shape, 16)
    std = psatd.coefficients(ks, dt)
    v = 1e-7
    gc = psatd.galilean_coefficients(ks, kc, (0.0, 0.0, v), dt)
    # first-order in v: |coefficient - standard| <= a few v dt |[k]_c| times the coefficient scale
    for g, s in (("TC", "C"), ("TS", "S_over_w"), ("X1", "X1"), ("X2", "X2"), ("TX3", "X3"), ("X4", "X4")):
        scale = np.max(np.abs(std[s])) + 1e-300
        assert np.max(np.abs(gc[g] - std[s])) <= 1e-5 * scale, g


@pytest.mark.parametrize("v", [(0.0, 0.0, -0.999), (0.3, -0.4, 0.5)])
def test_vacuum_update_eigenvalues_are_the_galilean_dispersion(v):
    """App. B: vacuum (transverse) modes advance by exp(i (W_c -+ w_s) dt) per step, i.e.
    w = c [k]_s + v_gal . (k - [k]_c) in the lab frame.  The two longitudinal directions, which
    the update leaves to the charge terms (Gauss's law), are scaled by theta^2 C."""
    shape, dt = (8, 8, 16), 0.7
    ks, kc = _grid_k(shape, 8)
    gc = psatd.galilean_coefficients(ks, kc, v, dt)
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    kcx, kcy, kcz = np.broadcast_arrays(*kc)
    rng = np.random.default_rng(3)
    for _ in range(12):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        kvec = [np.array(ksx[idx]), np.array(ksy[idx]), np.array(ksz[idx])]
        g = {k: np.array(val[idx]) for k, val in gc.items()}
        M = np.zeros((6, 6), dtype=complex)
        z = np.array(0j)
        for col in range(6):
            x = [np.array(0j) for _ in range(6)]
            x[col] = np.array(1 + 0j)
            E, B = psatd.update_galilean(x[:3], x[3:], [z, z, z], z, z, kvec, g)
            M[:, col] = [complex(a) for a in list(E) + list(B)]
        ws = np.sqrt(sum(float(a) ** 2 for a in kvec))
        W = v[0] * float(kcx[idx]) + v[1] * float(kcy[idx]) + v[2] * float(kcz[idx])
        expect = np.exp(1j * W * dt) * np.array([np.exp(-1j * ws * dt)] * 2 + [np.exp(1j * ws * dt)] * 2
                                                + [np.cos(ws * dt)] * 2)
        got = np.linalg.eigvals(M)
        for e in expect:  # each expected eigenvalue is found (multiplicities by greedy matching)
            i = int(np.argmin(np.abs(got - e)))
            assert abs(got[i] - e) <= 1e-9, (idx, e, got)
            got = np.delete(got, i)


def _ode_step(ks, W, E0, B0, J, dt):
    """Integrates (d/dt - i W) B = -i ks x E, (d/dt - i W) E = i ks x B - J (c = eps0 = 1) over dt."""
    def rhs(t, y):
        z = y[:6] + 1j * y[6:]
        E, B = z[:3], z[3:]
        dB = 1j * W * B - 1j * np.cross(ks, E)
        dE = 1j * W * E + 1j * np.cross(ks, B) - J
        d = np.concatenate([dE, dB])
        return np.concatenate([d.real, d.imag])
    z0 = np.concatenate([E0, B0])
    sol = solve_ivp(rhs, (0.0, dt), np.concatenate([z0.real, z0.imag]), method="DOP853", rtol=1e-13, atol=1e-15)
    y = sol.y[:, -1]
    z = y[:6] + 1j * y[6:]
    return z[:3], z[3:]


@pytest.mark.parametrize("order,v", [(16, (0.0, 0.0, -0.999)), (4, (0.2, 0.6, -0.5))])
def test_update_integrates_the_galilean_maxwell_equations(order, v):
    shape, dt = (8, 8, 16), 0.5
    ks, kc = _grid_k(shape, order)
    gc = psatd.galilean_coefficients(ks, kc, v, dt)
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    kcx, kcy, kcz = np.broadcast_arrays(*kc)
    rng = np.random.default_rng(4)
    for _ in range(16):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        k = np.array([ksx[idx], ksy[idx], ksz[idx]], dtype=float)
        W = v[0] * kcx[idx] + v[1] * kcy[idx] + v[2] * kcz[idx]
        E0 = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        B0 = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        if np.dot(k, k) > 0:
            B0 = B0 - k * np.dot(k, B0) / np.dot(k, k)  # div B = 0
        J = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        rho0 = 1j * np.dot(k, E0)  # Gauss: [k]_s . E = -i rho
        # Galilean continuity (d/dt - i W) rho + i [k]_s . J = 0, solved exactly over the step
        kJ = np.dot(k, J)
        rho1 = np.exp(1j * W * dt) * rho0 + (-1j * kJ) * ((np.exp(1j * W * dt) - 1) / (1j * W) if W != 0 else dt)
        g = {key: np.array(val[idx]) for key, val in gc.items()}
        kv = [np.array(x) for x in k]
        E1, B1 = psatd.update_galilean([np.array(x) for x in E0], [np.array(x) for x in B0],
                                       [np.array(x) for x in J], np.array(rho0), np.array(rho1), kv, g)
        Er, Br = _ode_step(k, W, E0, B0, J, dt)
        scale = np.max(np.abs(np.concatenate([Er, Br]))) + 1
        assert np.max(np.abs(np.array([complex(x) for x in E1]) - Er)) <= 1e-9 * scale, idx
        assert np.max(np.abs(np.array([complex(x) for x in B1]) - Br)) <= 1e-9 * scale, idx
        # Gauss's law carried to n+1
        assert abs(np.dot(k, np.array([complex(x) for x in E1])) + 1j * rho1) <= 1e-10 * scale


def test_particle_at_rest_drifts_backwards_in_the_galilean_frame():
    """A particle at rest in the lab, with no fields, moves by -v_gal dt per step on the grid
    that travels with v_gal (and deposits no current)."""
    from oracle.step import Params, step
    shape = (8, 8, 16)
    v = (0.0, 0.0, -0.6)
    p = Params(shape, (1.0, 1.0, 1.0), 0.5, 3, 4, 8, v_gal=v)
    zero = np.zeros(shape)
    st = {"E_stag": [zero.copy() for _ in range(3)], "B_stag": [zero.copy() for _ in range(3)],
          "rho_old": zero.copy()}
    pos0 = np.array([[1.25, 2.5, 3.75], [7.9, 0.1, 15.95]])
    sp = {"pos": pos0.copy(), "u": np.zeros((2, 3)), "w": np.ones(2), "q": -1.0, "m": 1.0}
    out = step(st, [sp], p)
    expect = np.mod(pos0 - 0.5 * np.asarray(v)[None, :], np.asarray(shape, dtype=float)[None, :])
    np.testing.assert_allclose(sp["pos"], expect, atol=1e-14)
    assert max(np.max(np.abs(j)) for j in out["J_nod"]) == 0.0


def test_extended_precision_branch_agrees_with_float64_closed_forms():
    """Where the float64 closed forms are still accurate (|W dt| ~ 0.1), the 40-digit evaluation
    used below |W dt| = 0.05 gives the same coefficients."""
    k = (0.7, -0.3, 0.2)
    for W in (0.1, 0.2, -0.3):
        dt = 0.5
        mp = psatd._galilean_mp(*k, W, dt)
        ks = tuple(np.array([x]) for x in k)
        kc = (np.array([W]), np.array([0.0]), np.array([0.0]))  # W = v . [k]_c with v = (1, 0, 0)
        gc = psatd.galilean_coefficients(ks, kc, (1.0, 0.0, 0.0), dt)
        for key, val in mp.items():
            assert abs(complex(gc[key][0]) - val) <= 1e-12 * (abs(val) + 1e-3), key


# ---------------------------------------------------------------- averaged Galilean PSATD (Sec. 4.4)

def _ode_average(ks, W, E0, B0, J, dt):
    """Mean over [dt/2, 3 dt/2] of the exact solution of the Galilean Fourier-space Maxwell
    equations (c = eps0 = 1) from (E0, B0) with constant J: the state is integrated to dt/2, then
    together with its running integral to 3 dt/2."""
    def rhs(t, y, acc):
        z = y[:6] + 1j * y[6:12]
        E, B = z[:3], z[3:]
        dB = 1j * W * B - 1j * np.cross(ks, E)
        dE = 1j * W * E + 1j * np.cross(ks, B) - J
        d = np.concatenate([dE, dB])
        out = np.concatenate([d.real, d.imag])
        if acc:
            out = np.concatenate([out, y[:12] / dt])
        return out
    z0 = np.concatenate([E0, B0])
    y0 = np.concatenate([z0.real, z0.imag])
    s1 = solve_ivp(lambda t, y: rhs(t, y, False), (0.0, dt / 2), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    y1 = np.concatenate([s1.y[:, -1], np.zeros(12)])
    s2 = solve_ivp(lambda t, y: rhs(t, y, True), (dt / 2, 1.5 * dt), y1, method="DOP853", rtol=1e-13, atol=1e-15)
    a = s2.y[12:, -1]
    z = a[:6] + 1j * a[6:]
    return z[:3], z[3:]


@pytest.mark.parametrize("order,v", [(16, (0.0, 0.0, -0.999)), (4, (0.2, 0.6, -0.5)), (8, (0.0, 0.0, 0.0))])
def test_averaged_update_is_the_mean_of_the_exact_solution(order, v):
    """Sec. 4.4: <E>, <B> equal the mean of the step's exact solution (same J) over
    [t_n + dt/2, t_n + 3 dt/2], with Gauss-consistent data and the Galilean continuity equation
    (a high-accuracy ODE integration), including k = 0 and W = 0 modes."""
    shape, dt = (8, 8, 16), 0.5
    ks, kc = _grid_k(shape, order)
    ac = psatd.averaged_coefficients(ks, kc, v, dt)
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    kcx, kcy, kcz = np.broadcast_arrays(*kc)
    rng = np.random.default_rng(5)
    picks = [(0, 0, 0), (1, 0, 0), (0, 0, 8)] + [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(14)]
    for idx in picks:
        k = np.array([ksx[idx], ksy[idx], ksz[idx]], dtype=float)
        W = v[0] * kcx[idx] + v[1] * kcy[idx] + v[2] * kcz[idx]
        W = 0.0 if abs(W * dt) < 1e-12 else W
        E0 = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        B0 = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        if np.dot(k, k) > 0:
            B0 = B0 - k * np.dot(k, B0) / np.dot(k, k)
        J = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        rho0 = 1j * np.dot(k, E0)
        kJ = np.dot(k, J)
        rho1 = np.exp(1j * W * dt) * rho0 + (-1j * kJ) * ((np.exp(1j * W * dt) - 1) / (1j * W) if W != 0 else dt)
        g = {key: np.array(val[idx]) for key, val in ac.items()}
        kv = [np.array(x) for x in k]
        Ea, Ba = psatd.update_averaged([np.array(x) for x in E0], [np.array(x) for x in B0],
                                       [np.array(x) for x in J], np.array(rho0), np.array(rho1), kv, g)
        Er, Br = _ode_average(k, W, E0, B0, J, dt)
        scale = np.max(np.abs(np.concatenate([Er, Br]))) + 1
        assert np.max(np.abs(np.array([complex(x) for x in Ea]) - Er)) <= 1e-9 * scale, idx
        assert np.max(np.abs(np.array([complex(x) for x in Ba]) - Br)) <= 1e-9 * scale, idx


def test_averaged_coefficients_without_galilean_velocity():
    """v_gal = 0: the means of cos(w t), -sin(w t)/w and (1 - cos(w t))/w^2 over [dt/2, 3 dt/2]."""
    shape, dt = (8, 12, 16), 0.7
    ks, kc = _grid_k(shape, 16)
    ac = psatd.averaged_coefficients(ks, kc, (0.0, 0.0, 0.0), dt)
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    w = np.sqrt(ksx ** 2 + ksy ** 2 + ksz ** 2)
    big = w * dt > 0.3
    wb = w[big]
    P1 = (np.sin(1.5 * wb * dt) - np.sin(0.5 * wb * dt)) / (wb * dt)
    P2 = (np.cos(1.5 * wb * dt) - np.cos(0.5 * wb * dt)) / (wb * wb * dt)
    np.testing.assert_allclose(ac["Psi1"][big], P1, atol=1e-13)
    np.testing.assert_allclose(ac["Psi2"][big], P2, atol=1e-13)
    np.testing.assert_allclose(ac["Y1"][big], (1 - P1) / wb ** 2, atol=1e-13)
    np.testing.assert_allclose(ac["Y4"][big], P2, atol=1e-13)
