"""Fornberg coefficients and modified wave numbers (oracle).

Test infrastructure only (see ``oracle/__init__``).

* staggered coefficients alpha^s_{m,n}: Sec. 3 (definition after eq.
  ``staggered_finite_difference``) and Sec. 4.1 eq. ``eq_Fornberg_staggered``;
* centered coefficients alpha^c_{m,n}: Sec. 4.1 eq. ``eq_Fornberg_centered``;
* modified wave numbers [k]_s and [k]_c: Sec. 4.1 eqs.
  ``staggered_modified_wave_number`` and ``centered_modified_wave_number``.

The coefficients are computed as exact rationals with ``fractions.Fraction``.
"""

from fractions import Fraction
from math import factorial

import numpy as np


def alpha_staggered(m):
    """alpha^s_{m,n} for n = 1..m as exact Fractions (order 2m).

    (-1)^(n+1) [ (2m)! / (2^(2m) m!) ]^2 * 4 / ((2n-1) (m-n)! (m+n-1)!)
    """
    if m < 1:
        raise ValueError("m must be >= 1")
    pref = Fraction(factorial(2 * m), 2 ** (2 * m) * factorial(m)) ** 2
    return [
        (-1) ** (n + 1) * pref * Fraction(4, (2 * n - 1) * factorial(m - n) * factorial(m + n - 1))
        for n in range(1, m + 1)
    ]


def alpha_centered(m):
    """alpha^c_{m,n} for n = 1..m as exact Fractions: (-1)^(n+1) 2 (m!)^2 / ((m-n)! (m+n)!)."""
    if m < 1:
        raise ValueError("m must be >= 1")
    return [
        (-1) ** (n + 1) * Fraction(2 * factorial(m) ** 2, factorial(m - n) * factorial(m + n))
        for n in range(1, m + 1)
    ]


def k_axis(n, d):
    """Grid wave numbers 2*pi*fftfreq(n, d) of an n-point periodic axis of spacing d.

    For even n the Nyquist index n/2 carries k = -pi/d (NumPy's convention)."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d)


def k_staggered(k, d, order):
    """Staggered modified wave number [k]_s at finite order 2m (``order``); order 0 = infinite.

    [k]_s = sum_n alpha^s_{m,n} sin(k (n-1/2) d) / ((n-1/2) d)
    """
    k = np.asarray(k, dtype=np.float64)
    if order == 0:
        return k.copy()
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2 (or 0 for infinite)")
    m = order // 2
    a = alpha_staggered(m)
    out = np.zeros_like(k)
    for n in range(1, m + 1):
        h = (n - 0.5) * d
        out += float(a[n - 1]) * np.sin(k * h) / h
    return out


def k_centered(k, d, order):
    """Centered modified wave number [k]_c = sum_n alpha^c_{m,n} sin(k n d)/(n d); order 0 = infinite."""
    k = np.asarray(k, dtype=np.float64)
    if order == 0:
        return k.copy()
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2 (or 0 for infinite)")
    m = order // 2
    a = alpha_centered(m)
    out = np.zeros_like(k)
    for n in range(1, m + 1):
        out += float(a[n - 1]) * np.sin(k * n * d) / (n * d)
    return out


def centering_transfer(k, d, m):
    """zeta_F(k) = sum_n alpha^s_{m,n} cos(k (n-1/2) d): Fourier multiplier of the centering (App. C)."""
    k = np.asarray(k, dtype=np.float64)
    a = alpha_staggered(m)
    out = np.zeros_like(k)
    for n in range(1, m + 1):
        out += float(a[n - 1]) * np.cos(k * (n - 0.5) * d)
    return out
