"""Pins of the oracle's particle operations.

* B-spline shapes: partition of unity, reproduction of linear functions, and the
  cubic spline against its truncated-power (divided difference) form;
* gather reproduces linear fields exactly; deposition conserves total charge and is
  the adjoint of gather;
* Boris: exact gyration angle 2 atan(|q| B dt / (2 m gamma)) and |u| conservation in a
  uniform B; exact du = q E dt / m in a uniform E; E x B drift velocity.
"""

from math import comb

import numpy as np
import pytest

from oracle import particles


@pytest.mark.parametrize("order", [1, 3])
def test_shape_partition_and_linear(order):
    x = np.random.default_rng(0).uniform(-5, 5, 1000)
    i0 = np.floor(x).astype(int)
    offs = (0, 1) if order == 1 else (-1, 0, 1, 2)
    w = [particles.shape_1d(order, x - (i0 + o)) for o in offs]
    np.testing.assert_allclose(sum(w), 1.0, atol=1e-14)
    np.testing.assert_allclose(sum(wi * (i0 + o) for wi, o in zip(w, offs)), x, atol=1e-13)
    # the support is complete: nodes outside contribute nothing
    far = [particles.shape_1d(order, x - (i0 + o)) for o in ((-1, 2) if order == 1 else (-2, 3))]
    assert np.all(np.abs(far[0]) < 1e-15) and np.all(np.abs(far[1]) < 1e-15)


def test_cubic_truncated_power_form():
    # centred cubic B-spline = (1/6) sum_j (-1)^j C(4,j) (d + 2 - j)_+^3
    d = np.linspace(-2.5, 2.5, 1001)
    tp = sum((-1) ** j * comb(4, j) * np.maximum(d + 2 - j, 0) ** 3 for j in range(5)) / 6
    np.testing.assert_allclose(particles.shape_1d(3, d), tp, atol=1e-13)
    lin = np.maximum(1 - np.abs(d), 0)
    np.testing.assert_allclose(particles.shape_1d(1, d), lin, atol=1e-15)


@pytest.mark.parametrize("order", [1, 3])
def test_gather_linear_field_exact(order):
    shape, spacing = (24, 20, 28), (1.0, 0.5, 2.0)
    X, Y, Z = np.meshgrid(*[np.arange(n) * d for n, d in zip(shape, spacing)], indexing="ij")
    F = 0.3 + 0.7 * X - 1.1 * Y + 0.2 * Z
    rng = np.random.default_rng(2)
    lo = np.array([4, 4, 4]) * spacing
    hi = (np.array(shape) - 5) * np.array(spacing)
    pos = rng.uniform(lo, hi, (500, 3))
    got = particles.gather([F], pos, spacing, order)[0]
    np.testing.assert_allclose(got, 0.3 + 0.7 * pos[:, 0] - 1.1 * pos[:, 1] + 0.2 * pos[:, 2], atol=1e-12)


@pytest.mark.parametrize("order", [1, 3])
def test_deposit_charge_and_adjoint(order):
    shape, spacing = (8, 6, 10), (1.0, 0.5, 2.0)
    L = np.array(shape) * np.array(spacing)
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 1, (300, 3)) * L
    q = rng.standard_normal(300)
    rho = particles.deposit([q], pos, shape, spacing, order)[0]
    dV = np.prod(spacing)
    assert np.sum(rho) * dV == pytest.approx(np.sum(q), rel=1e-13)
    F = rng.standard_normal(shape)
    assert np.sum(rho * F) * dV == pytest.approx(np.sum(q * particles.gather([F], pos, spacing, order)[0]), rel=1e-12)


def test_boris_gyration_exact():
    B0, q, m, dt = 0.8, -1.0, 1.0, 0.5
    u = np.array([[0.3], [0.4], [0.1]])
    E = np.zeros((3, 1))
    B = np.array([[0.0], [0.0], [B0]])
    g = particles.gamma(u)[0]
    theta = 2 * np.arctan(abs(q) * B0 * dt / (2 * m * g))
    ang0 = np.arctan2(u[1, 0], u[0, 0])
    for n in range(1, 30):
        u = particles.boris(u, E, B, q, m, dt)
        assert np.linalg.norm(u) == pytest.approx(np.sqrt(0.3 ** 2 + 0.4 ** 2 + 0.1 ** 2), rel=1e-14)
        ang = np.arctan2(u[1, 0], u[0, 0])
        # an electron (q < 0) gyrates counter-clockwise about +z
        expect = ang0 + n * theta
        assert np.angle(np.exp(1j * (ang - expect))) == pytest.approx(0.0, abs=1e-12)
        assert u[2, 0] == pytest.approx(0.1, abs=1e-15)


def test_boris_uniform_electric():
    u = np.array([[0.1], [-0.2], [0.05]])
    E = np.array([[0.3], [0.1], [-0.7]])
    q, m, dt = -1.0, 2.0, 0.4
    u1 = particles.boris(u, E, np.zeros((3, 1)), q, m, dt)
    np.testing.assert_allclose(u1, u + q * E * dt / m, atol=1e-15)


def test_boris_exb_drift():
    # Non-relativistic E x B drift: mean velocity E x B / |B|^2.
    E = np.array([[0.0], [1e-4], [0.0]])
    B = np.array([[0.0], [0.0], [0.5]])
    u = np.zeros((3, 1))
    q, m, dt = -1.0, 1.0, 0.1
    period = 2 * np.pi * m / (abs(q) * 0.5)
    nper = 20
    n = int(round(nper * period / dt))
    vs = []
    for _ in range(n):
        u = particles.boris(u, E, B, q, m, dt)
        vs.append(u[:, 0] / particles.gamma(u)[0])
    vmean = np.mean(vs, axis=0)
    drift = np.cross(E[:, 0], B[:, 0]) / 0.25
    assert vmean[0] == pytest.approx(drift[0], rel=0.02)
    assert abs(vmean[1]) < 0.02 * abs(drift[0])
