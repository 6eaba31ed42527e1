"""Pins of the oracle's Fornberg coefficients, modified wave numbers and PSATD coefficients.

Each pin compares the oracle with an independent derivation: Lagrange
interpolation/differentiation weights computed from their own definition,
the finite-difference stencil applied to a sampled exponential, closed-form
limits, and an extended-precision evaluation.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import fornberg, psatd


def lagrange_weights_at0(nodes):
    """Interpolation weights L_i(0) for the given exact nodes."""
    w = []
    for i, xi in enumerate(nodes):
        p = Fraction(1)
        for k, xk in enumerate(nodes):
            if k != i:
                p *= (0 - xk) / (xi - xk)
        w.append(p)
    return w


def lagrange_derivative_at0(nodes):
    """Differentiation weights L_i'(0)."""
    w = []
    for i, xi in enumerate(nodes):
        tot = Fraction(0)
        for k, xk in enumerate(nodes):
            if k == i:
                continue
            p = Fraction(1, 1) / (xi - xk)
            for l, xl in enumerate(nodes):
                if l != i and l != k:
                    p *= (0 - xl) / (xi - xl)
            tot += p
        w.append(tot)
    return w


@pytest.mark.parametrize("m", list(range(1, 17)))
def test_staggered_alpha_is_midpoint_lagrange(m):
    # Sec. 3: the centering sum with alpha^s/2 must be 2m-point interpolation at the midpoint.
    a = fornberg.alpha_staggered(m)
    nodes = [Fraction(2 * n - 1, 2) for n in range(1, m + 1)] + [Fraction(-(2 * n - 1), 2) for n in range(1, m + 1)]
    L = lagrange_weights_at0(nodes)
    for n in range(1, m + 1):
        assert a[n - 1] / 2 == L[n - 1] == L[m + n - 1]


@pytest.mark.parametrize("m", list(range(1, 11)))
def test_staggered_alpha_is_midpoint_derivative(m):
    # Sec. 3 eq. staggered_finite_difference: weight of f_{n-1/2} is alpha^s_{m,n}/(2n-1).
    a = fornberg.alpha_staggered(m)
    nodes = [Fraction(2 * n - 1, 2) for n in range(1, m + 1)] + [Fraction(-(2 * n - 1), 2) for n in range(1, m + 1)]
    D = lagrange_derivative_at0(nodes)
    for n in range(1, m + 1):
        assert a[n - 1] / (2 * n - 1) == D[n - 1] == -D[m + n - 1]


@pytest.mark.parametrize("m", list(range(1, 11)))
def test_centered_alpha_is_central_derivative(m):
    # Sec. 4.1 / App. A: centered difference weight of f_n is alpha^c_{m,n}/(2n).
    a = fornberg.alpha_centered(m)
    nodes = [Fraction(0)] + [Fraction(n) for n in range(1, m + 1)] + [Fraction(-n) for n in range(1, m + 1)]
    D = lagrange_derivative_at0(nodes)
    assert D[0] == 0
    for n in range(1, m + 1):
        assert a[n - 1] / (2 * n) == D[n] == -D[m + n]


def test_textbook_values():
    assert fornberg.alpha_staggered(1) == [1]
    assert fornberg.alpha_staggered(2) == [Fraction(9, 8), Fraction(-1, 8)]
    assert fornberg.alpha_centered(1) == [1]
    assert fornberg.alpha_centered(2) == [Fraction(4, 3), Fraction(-1, 3)]


@pytest.mark.parametrize("m", [1, 2, 3, 4, 8, 16])
def test_fornberg_moments(m):
    # eq. eq_Fornberg_property.  Reading: the moments vanish for k = 1..m-1; the k = m moment does not.
    a = fornberg.alpha_staggered(m)
    mom = lambda k: sum(a[n - 1] * Fraction(2 * n - 1, 2) ** (2 * k) for n in range(1, m + 1))
    assert mom(0) == 1
    for k in range(1, m):
        assert mom(k) == 0
    assert mom(m) != 0


@pytest.mark.parametrize("order", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("d", [1.0, 0.7])
def test_staggered_wavenumber_is_stencil_eigenvalue(order, d):
    # App. A eq. staggered_finite_difference_nodal: the nodal->centre staggered difference of
    # exp(i k x) equals i [k]_s exp(i k x_{j+1/2}).
    m = order // 2
    a = fornberg.alpha_staggered(m)
    N = 64
    k = fornberg.k_axis(N, d)
    j = np.arange(N)
    for kk in k[1:]:
        f = np.exp(1j * kk * j * d)
        fd = sum(float(a[n - 1]) * (np.roll(f, -n) - np.roll(f, n - 1)) / ((2 * n - 1) * d) for n in range(1, m + 1))
        expect = 1j * fornberg.k_staggered(kk, d, order) * np.exp(1j * kk * (j + 0.5) * d)
        np.testing.assert_allclose(fd, expect, atol=1e-12 * (1 + abs(kk)))


@pytest.mark.parametrize("order", [2, 4, 16])
def test_centered_wavenumber_is_stencil_eigenvalue(order):
    m = order // 2
    a = fornberg.alpha_centered(m)
    N, d = 48, 1.0
    j = np.arange(N)
    for kk in fornberg.k_axis(N, d)[1:]:
        f = np.exp(1j * kk * j * d)
        fd = sum(float(a[n - 1]) * (np.roll(f, -n) - np.roll(f, n)) / (2 * n * d) for n in range(1, m + 1))
        np.testing.assert_allclose(fd, 1j * fornberg.k_centered(kk, d, order) * f, atol=1e-12)


def test_order2_is_yee_and_infinite_is_exact():
    k = fornberg.k_axis(32, 1.0)
    np.testing.assert_allclose(fornberg.k_staggered(k, 1.0, 2), 2 * np.sin(k / 2), atol=1e-15)
    np.testing.assert_array_equal(fornberg.k_staggered(k, 1.0, 0), k)
    # high order converges to k away from Nyquist
    kk = k[np.abs(k) < 2.0]
    assert np.max(np.abs(fornberg.k_staggered(kk, 1.0, 64) - kk)) < 1e-6


def test_psatd_coefficient_limits_at_k0():
    dt = 0.37
    z = np.zeros(1)
    c = psatd.coefficients((z, z, z), dt)
    assert c["C"][0] == 1.0
    assert c["S_over_w"][0] == pytest.approx(dt, rel=1e-15)
    assert c["X1"][0] == pytest.approx(dt ** 2 / 2, rel=1e-15)
    assert c["X2"][0] == pytest.approx(dt ** 2 / 6, rel=1e-15)
    assert c["X3"][0] == pytest.approx(-dt ** 2 / 3, rel=1e-15)
    assert c["X4"][0] == pytest.approx(-dt, rel=1e-15)


def test_psatd_coefficients_extended_precision():
    # Definitions of Sec. 4.2 evaluated directly in 80-bit extended precision.
    dt = 0.5
    w = np.concatenate([np.geomspace(1e-3, 0.2, 40), np.linspace(0.2, 12.0, 40)])
    c = psatd.coefficients((w, np.zeros_like(w), np.zeros_like(w)), dt)
    wl = w.astype(np.longdouble)
    xl = wl * np.longdouble(dt)
    Cl, Sl = np.cos(xl), np.sin(xl)
    ref = {
        "C": Cl, "S_over_w": Sl / wl, "X1": (1 - Cl) / wl ** 2,
        "X2": (1 - Sl / xl) / wl ** 2, "X3": (Cl - Sl / xl) / wl ** 2, "X4": -Sl / wl,
    }
    # the extended-precision reference itself cancels in (1 - C), (1 - S/x), (C - S/x): ~1e-19/x^2 relative
    tol = 5e-14 + 1e-18 / (w * dt) ** 2
    for key, r in ref.items():
        r = r.astype(np.float64)
        err = np.abs(c[key] - r) / np.abs(r)
        assert np.all(err <= tol), (key, float(np.max(err / tol)))


def test_golden_fornberg_table():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fornberg_staggered.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    for m, n, num, den in rows:
        assert fornberg.alpha_staggered(int(m))[int(n) - 1] == Fraction(int(num), int(den))
    # textbook midpoint weights of the 6-point rule: 150/256, -25/256, 3/256 (times 2)
    assert fornberg.alpha_staggered(3) == [Fraction(75, 64), Fraction(-25, 128), Fraction(3, 128)]
