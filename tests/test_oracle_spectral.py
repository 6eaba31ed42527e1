"""Pins of the oracle's Fourier convention and standard-PSATD update.

* the paper-convention transform against a brute-force DFT with explicit positions;
* the per-mode update against the matrix exponential of the k-space Maxwell curl
  equations (the update integrates them exactly when Gauss's law and continuity hold);
* vacuum plane waves advance by exactly w_s = c|[k]_s| per unit time (App. B);
* Gauss's law is preserved, the k = 0 mode is a pure current drive, the vacuum update
  is time-reversible (App. B).
"""

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import dft, fornberg, psatd, transforms
from oracle.step import Params, push_fields
from oracle.transforms import OFFSETS


@pytest.mark.parametrize("shape", [(3, 4, 6), (4, 2, 3), (6, 5, 2)])
@pytest.mark.parametrize("name", ["rho", "Ex", "Ey", "Ez", "Bx", "By", "Bz"])
def test_forward_matches_naive_dft(shape, name):
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape)
    spacing = (1.0, 0.8, 1.3)
    got = transforms.forward(f, spacing, OFFSETS[name])
    ref = dft.naive_forward(f, spacing, OFFSETS[name])
    np.testing.assert_allclose(got, ref, atol=1e-12)
    back = transforms.inverse(got, spacing, OFFSETS[name])
    np.testing.assert_allclose(back, f, atol=1e-13)
    # Parseval
    assert np.sum(np.abs(got) ** 2) == pytest.approx(f.size * np.sum(f ** 2), rel=1e-13)


def _mode_setup(rng, K):
    """Random Gauss-consistent mode: returns E, B (div-free), J, rho_old, rho_new for dt."""
    E = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    B = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    J = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    K2 = K @ K
    B = B - K * (K @ B) / K2
    return E, B, J


@pytest.mark.parametrize("seed", range(6))
def test_update_equals_exact_integration(seed):
    # The update of Sec. 4.2 integrates dB/dt = -i K x E, dE/dt = i c^2 K x B - J/eps0 exactly
    # (J constant over the step) when rho^n = i eps0 K.E^n and rho^{n+1} follows continuity.
    rng = np.random.default_rng(seed)
    K = rng.standard_normal(3) * rng.uniform(0.1, 3.0)
    dt = rng.uniform(0.1, 2.5)
    E, B, J = _mode_setup(rng, K)
    rho_old = 1j * (K @ E)
    rho_new = rho_old - 1j * dt * (K @ J)
    coef = psatd.coefficients(tuple(np.array([k]) for k in K), dt)
    coef = {k: v[0] for k, v in coef.items()}
    E1, B1 = psatd.update(tuple(E), tuple(B), tuple(J), rho_old, rho_new, tuple(K), coef)

    def crossmat(v):
        return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]], dtype=complex)

    A = np.zeros((7, 7), dtype=complex)
    A[0:3, 3:6] = 1j * crossmat(K)       # dE/dt = i K x B - J
    A[0:3, 6] = -J
    A[3:6, 0:3] = -1j * crossmat(K)      # dB/dt = -i K x E
    y = expm(A * dt) @ np.concatenate([E, B, [1.0]])
    np.testing.assert_allclose(np.array(E1), y[0:3], atol=1e-12 * (1 + np.abs(y).max()))
    np.testing.assert_allclose(np.array(B1), y[3:6], atol=1e-12 * (1 + np.abs(y).max()))


def test_gauss_preserved_and_violation_scaled():
    rng = np.random.default_rng(11)
    for _ in range(20):
        K = rng.standard_normal(3)
        dt = rng.uniform(0.1, 2.0)
        E, B, J = _mode_setup(rng, K)
        rho_old = 1j * (K @ E)
        R = rng.standard_normal() + 1j * rng.standard_normal()   # continuity violation
        rho_new = rho_old - 1j * dt * (K @ J) + dt * R
        coef = {k: v[0] for k, v in psatd.coefficients(tuple(np.array([k]) for k in K), dt).items()}
        E1, B1 = psatd.update(tuple(E), tuple(B), tuple(J), rho_old, rho_new, tuple(K), coef)
        E1, B1 = np.array(E1), np.array(B1)
        assert abs(K @ B1) < 1e-12
        # new Gauss residual K.E + i rho_new equals (S/w)-scaled violation: i X2 |K|^2 dt R ... closed form
        res = K @ E1 + 1j * rho_new
        w = np.sqrt(K @ K)
        expect = 1j * dt * R * (1 - coef["X2"] * w ** 2)   # = i dt R S/(w dt)
        assert abs(res - expect) < 1e-12 * (1 + abs(expect))
        assert abs(expect - 1j * R * np.sin(w * dt) / w) < 1e-12


def test_k0_mode_is_current_drive():
    rng = np.random.default_rng(5)
    E, B, J = (rng.standard_normal(3) + 0j for _ in range(3))
    z = (0.0, 0.0, 0.0)
    dt = 0.7
    coef = {k: v[0] for k, v in psatd.coefficients(tuple(np.array([k]) for k in z), dt).items()}
    E1, B1 = psatd.update(tuple(E), tuple(B), tuple(J), 0.3, -0.2, z, coef)
    np.testing.assert_allclose(np.array(E1), E - dt * J, atol=1e-15)
    np.testing.assert_allclose(np.array(B1), B, atol=1e-15)


def test_vacuum_time_reversal():
    # App. B: swapping n <-> n+1 and flipping the sign of B inverts the vacuum update.
    rng = np.random.default_rng(9)
    K = rng.standard_normal(3)
    E, B, _ = _mode_setup(rng, K)
    E = E - K * (K @ E) / (K @ K)      # vacuum: no charge, so E is transverse too
    z3 = (0j, 0j, 0j)
    dt = 1.3
    coef = {k: v[0] for k, v in psatd.coefficients(tuple(np.array([k]) for k in K), dt).items()}
    E1, B1 = psatd.update(tuple(E), tuple(B), z3, 0j, 0j, tuple(K), coef)
    E0, mB0 = psatd.update(E1, tuple(-np.array(B1)), z3, 0j, 0j, tuple(K), coef)
    np.testing.assert_allclose(np.array(E0), E, atol=1e-13)
    np.testing.assert_allclose(-np.array(mB0), B, atol=1e-13)


@pytest.mark.parametrize("order", [2, 16, 0])
def test_vacuum_plane_wave_dispersion(order):
    # App. B eq. vacuum_disprel_psatd: w = c [k]_s, for any dt (no stability limit).
    # Oblique wave k = (kx, ky, 0), E along z; B = [k]_s x E / w sampled at the B positions.
    shape, spacing, dt, nsteps = (16, 12, 4), (1.0, 1.0, 1.0), 1.7, 5
    kx = 2 * np.pi * 3 / 16
    ky = 2 * np.pi * 2 / 12
    Kx = fornberg.k_staggered(kx, 1.0, order)
    Ky = fornberg.k_staggered(ky, 1.0, order)
    w = np.hypot(Kx, Ky)

    def field(name, amp, t):
        o = OFFSETS[name]
        x = (np.arange(shape[0]) + o[0])[:, None, None]
        y = (np.arange(shape[1]) + o[1])[None, :, None]
        return amp * np.cos(kx * x + ky * y - w * t) * np.ones(shape)

    def state(t):
        E = [np.zeros(shape), np.zeros(shape), field("Ez", 1.0, t)]
        B = [field("Bx", Ky / w, t), field("By", -Kx / w, t), np.zeros(shape)]
        return E, B

    p = Params(shape, spacing, dt, 1, 2, order)
    E, B = state(0.0)
    zero = np.zeros(shape)
    for _ in range(nsteps):
        E, B = push_fields(E, B, [zero, zero, zero], zero, zero, p)
    Eref, Bref = state(nsteps * dt)
    for d in range(3):
        np.testing.assert_allclose(E[d], Eref[d], atol=1e-12)
        np.testing.assert_allclose(B[d], Bref[d], atol=1e-12)
