"""Pins of the oracle's finite-order centering (Sec. 3, App. C).

* a sampled sinusoid is an eigenfunction: centering multiplies it by
  zeta(k) = sum_n alpha^s_{m,n} cos(k (n-1/2) dx) (App. C), checked with an
  independent trigonometric evaluation;
* polynomials of degree <= 2m-1 are reproduced exactly, degree 2m is not
  (reading of the error order printed in Sec. 3);
* nodal->staggered and staggered->nodal are exact transposes;
* Fig. 4: I_n[I_s[f]] converges to f as the order grows.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import centering, fornberg


@pytest.mark.parametrize("m", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sinusoid_eigenfunction(m, axis):
    N = 40
    shape = [4, 4, 4]
    shape[axis] = N
    j = np.arange(N, dtype=np.float64)
    for kidx, phi in [(1, 0.3), (5, 1.1), (13, -0.4), (19, 0.0)]:
        k = 2 * np.pi * kidx / N
        zeta = fornberg.centering_transfer(k, 1.0, m)
        sl = [None, None, None]
        sl[axis] = slice(None)
        stag = np.broadcast_to(np.cos(k * (j + 0.5) + phi)[tuple(sl)], shape).copy()
        nod = np.broadcast_to(np.cos(k * j + phi)[tuple(sl)], shape).copy()
        np.testing.assert_allclose(centering.s2n_axis(stag, axis, m), zeta * nod, atol=1e-13)
        np.testing.assert_allclose(centering.n2s_axis(nod, axis, m), zeta * stag, atol=1e-13)


def test_transfer_error_order():
    # 1 - zeta(k) = O((k dx)^(2m)): halving k divides the error by ~4^m.
    for m in (1, 2, 4):
        e1 = 1 - fornberg.centering_transfer(0.2, 1.0, m)
        e2 = 1 - fornberg.centering_transfer(0.1, 1.0, m)
        assert e1 / e2 == pytest.approx(4 ** m, rel=0.02)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6])
def test_polynomial_exactness(m):
    # Exact rationals on a long periodic line; only interior nodes (far from the wrap) are checked.
    N = 64
    a = fornberg.alpha_staggered(m)
    for deg in range(0, 2 * m + 1):
        f = lambda x: Fraction(x) ** deg
        ok = True
        for j in range(m + 2, N - m - 2):
            s = sum(a[n - 1] * (f(Fraction(2 * j + 2 * n - 1, 2)) + f(Fraction(2 * j - 2 * n + 1, 2))) / 2
                    for n in range(1, m + 1))
            ok &= (s == f(j))
        assert ok == (deg <= 2 * m - 1)
        # and the oracle's float routine agrees with the exact evaluation on that polynomial
        stag = np.array([float(f(Fraction(2 * i + 1, 2))) for i in range(N)])[:, None, None] * np.ones((1, 2, 2))
        got = centering.s2n_axis(stag, 0, m)[m + 2:N - m - 2, 0, 0]
        if deg <= 2 * m - 1:
            ref = np.array([float(f(j)) for j in range(m + 2, N - m - 2)])
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("m", [1, 3, 8])
@pytest.mark.parametrize("name", ["Ex", "Ey", "Ez", "Bx", "By", "Bz"])
def test_n2s_is_transpose_of_s2n(m, name):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((10, 12, 18))
    y = rng.standard_normal((10, 12, 18))
    lhs = np.sum(centering.n2s(name, x, m) * y)
    rhs = np.sum(x * centering.s2n(name, y, m))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_fig4_round_trip_converges():
    # Fig. 4: f(x) = cos^5(4 pi x) and a binomially filtered Kronecker delta, orders 2, 4, 8, 16.
    N = 48
    x = np.arange(N) / N
    f = np.cos(4 * np.pi * x) ** 5
    delta = np.zeros(N)
    delta[N // 2] = 1.0
    delta = 0.25 * np.roll(delta, 1) + 0.5 * delta + 0.25 * np.roll(delta, -1)
    for sig in (f, delta):
        arr = sig[:, None, None] * np.ones((1, 2, 2))
        errs = []
        for order in (2, 4, 8, 16):
            m = order // 2
            back = centering.s2n_axis(centering.n2s_axis(arr, 0, m), 0, m)
            errs.append(np.max(np.abs(back - arr)))
        assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
