"""Standard PSATD on the staggered grid (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 4.1 (notation) and Sec. 4.2, eqs. ``eq_update_B_with_rho_standard`` and
``eq_update_E_with_rho_standard``:
    B^{n+1} = C B^n - i (S/w_s) [k]_s x E^n + i X1 [k]_s x J^{n+1/2}
    E^{n+1} = C E^n + i c^2 (S/w_s) [k]_s x B^n + X4 J^{n+1/2}
              + i (X3 rho^n - X2 rho^{n+1}) [k]_s
with w_s = c |[k]_s|, C = cos(w_s dt), S = sin(w_s dt) and
    X1 = (1 - C)/(eps0 w_s^2),  X2 = c^2 (1 - S/(w_s dt))/(eps0 w_s^2),
    X3 = c^2 (C - S/(w_s dt))/(eps0 w_s^2),  X4 = -S/(eps0 w_s).

The paper leaves w_s = 0 out ("assuming w_s != 0", end of Sec. 4.1).  Reading
used here: each coefficient takes its limit w_s -> 0 (S/w_s -> dt,
X1 -> dt^2/(2 eps0), X2 -> c^2 dt^2/(6 eps0), X3 -> -c^2 dt^2/(3 eps0),
X4 -> -dt/eps0).  Below w_s dt = 0.2 every coefficient is evaluated by the
Taylor series of its definition (eight terms; the same functions, free of the
cancellation in 1 - S/(w_s dt) and C - S/(w_s dt)); above it 1 - C is written
2 sin^2(w_s dt / 2).
"""

from math import factorial

import numpy as np

from .fornberg import k_centered, k_staggered
from .transforms import wave_vectors

C_LIGHT = 1.0
EPS0 = 1.0
SERIES_BELOW = 0.2


def staggered_wave_vector(shape, spacing, order):
    """([k^x]_s, [k^y]_s, [k^z]_s) as broadcastable 3D arrays."""
    kx, ky, kz = wave_vectors(shape, spacing)
    dx, dy, dz = spacing
    return (k_staggered(kx, dx, order), k_staggered(ky, dy, order), k_staggered(kz, dz, order))


def centered_wave_vector(shape, spacing, order):
    """([k^x]_c, [k^y]_c, [k^z]_c): the nodal solver's centered modified wave numbers (Sec. 4.1)."""
    kx, ky, kz = wave_vectors(shape, spacing)
    dx, dy, dz = spacing
    return (k_centered(kx, dx, order), k_centered(ky, dy, order), k_centered(kz, dz, order))


def _series(x2, coef):
    """sum_k coef[k] * x2**k (Horner)."""
    out = np.zeros_like(x2)
    for c in reversed(coef):
        out = out * x2 + c
    return out


# Taylor coefficients in x^2 (x = w_s dt), k = 0..7, from the sine and cosine series:
#   sin(x)/x            = sum_k (-1)^k x^(2k) / (2k+1)!
#   (1 - cos x)/x^2     = sum_k (-1)^k x^(2k) / (2k+2)!
#   (1 - sin(x)/x)/x^2  = sum_k (-1)^k x^(2k) / (2k+3)!
#   (cos x - sin(x)/x)/x^2 = sum_k (-1)^(k+1) x^(2k) (2k+2) / (2k+3)!
_SINC = [(-1) ** k / factorial(2 * k + 1) for k in range(8)]
_ONE_MINUS_COS = [(-1) ** k / factorial(2 * k + 2) for k in range(8)]
_ONE_MINUS_SINC = [(-1) ** k / factorial(2 * k + 3) for k in range(8)]
_COS_MINUS_SINC = [(-1) ** (k + 1) * (2 * k + 2) / factorial(2 * k + 3) for k in range(8)]


def coefficients(ks, dt):
    """C, S/w_s, X1, X2, X3, X4 on the (broadcast) grid of modified wave vectors ``ks``."""
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    w = C_LIGHT * np.sqrt(ksx ** 2 + ksy ** 2 + ksz ** 2)
    x = w * dt
    small = np.abs(x) < SERIES_BELOW  # |w dt|: the series serves a negative (time-reversed) dt too
    wsafe = np.where(small, 1.0, w)
    x2 = np.where(small, x * x, 0.0)

    C = np.cos(x)
    S = np.sin(x)
    S_over_w = np.where(small, dt * _series(x2, _SINC), S / wsafe)
    X1 = np.where(small, dt ** 2 * _series(x2, _ONE_MINUS_COS) / EPS0,
                  2.0 * np.sin(0.5 * x) ** 2 / (EPS0 * wsafe ** 2))
    X2 = np.where(small, C_LIGHT ** 2 * dt ** 2 * _series(x2, _ONE_MINUS_SINC) / EPS0,
                  C_LIGHT ** 2 * (1 - S / (wsafe * dt)) / (EPS0 * wsafe ** 2))
    X3 = np.where(small, C_LIGHT ** 2 * dt ** 2 * _series(x2, _COS_MINUS_SINC) / EPS0,
                  C_LIGHT ** 2 * (C - S / (wsafe * dt)) / (EPS0 * wsafe ** 2))
    X4 = -S_over_w / EPS0
    return {"C": C, "S_over_w": S_over_w, "X1": X1, "X2": X2, "X3": X3, "X4": X4}


def cross(a, b):
    """Component-wise cross product of two 3-lists of arrays."""
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def update(Eh, Bh, Jh, rho_old_h, rho_new_h, ks, coef):
    """One standard-PSATD step of the paper-convention spectra; returns (E_new, B_new) 3-tuples."""
    C, Sw = coef["C"], coef["S_over_w"]
    X1, X2, X3, X4 = coef["X1"], coef["X2"], coef["X3"], coef["X4"]
    kxE = cross(ks, Eh)
    kxB = cross(ks, Bh)
    kxJ = cross(ks, Jh)
    B_new = tuple(C * Bh[d] - 1j * Sw * kxE[d] + 1j * X1 * kxJ[d] for d in range(3))
    E_new = tuple(C * Eh[d] + 1j * C_LIGHT ** 2 * Sw * kxB[d] + X4 * Jh[d]
                  + 1j * (X3 * rho_old_h - X2 * rho_new_h) * ks[d] for d in range(3))
    return E_new, B_new


def update_transpose(lam_E, lam_B, ks, coef):
    """Conjugate transpose of ``update`` acting on the adjoint spectra (dL/dE', dL/dB').

    ``update`` is complex-linear in (E, B, J, rho^n, rho^{n+1}) with real coefficients and
    real [k]_s, so every term a * x of it contributes conj(a) * lambda to the adjoint of x,
    and a cross product [k]_s x v contributes -[k]_s x lambda.  Returns
    (gE, gB, gJ) 3-tuples and g_rho_old, g_rho_new."""
    C, Sw = coef["C"], coef["S_over_w"]
    X1, X2, X3, X4 = coef["X1"], coef["X2"], coef["X3"], coef["X4"]
    kxlE = cross(ks, lam_E)
    kxlB = cross(ks, lam_B)
    k_dot_lE = ks[0] * lam_E[0] + ks[1] * lam_E[1] + ks[2] * lam_E[2]
    gE = tuple(C * lam_E[d] - 1j * Sw * kxlB[d] for d in range(3))
    gB = tuple(C * lam_B[d] + 1j * C_LIGHT ** 2 * Sw * kxlE[d] for d in range(3))
    gJ = tuple(1j * X1 * kxlB[d] + X4 * lam_E[d] for d in range(3))
    return gE, gB, gJ, -1j * X3 * k_dot_lE, 1j * X2 * k_dot_lE


# ---------------------------------------------------------------- standard Galilean PSATD (Sec. 4.3)

def galilean_coefficients(ks, kc, v_gal, dt):
    """Per-mode coefficients of the standard Galilean update on the staggered grid (Sec. 4.1
    definitions, Sec. 4.3 eqs. ``eq_update_B/E_with_rho_galilean``):
      w_s = c |[k]_s|, w_c = c |[k]_c|, W = v_gal . [k]_c, C = cos(w_s dt), S = sin(w_s dt),
      theta = exp(i W dt / 2), chi1 = w_c^2 / (w_s^2 - W^2) (theta* - theta C + i W theta S / w_s),
      X1 = theta chi1 / (eps0 w_c^2),
      X2 = c^2 / (theta* - theta) (theta* X1 - theta (1 - C) / (eps0 w_s^2)),
      X3 = c^2 / (theta* - theta) (theta* X1 - theta* (1 - C) / (eps0 w_s^2)),
      X4 = i W X1 - theta^2 S / (eps0 w_s).
    Readings: w_c^2 cancels between chi1 and X1 (it vanishes at the Nyquist index of
    finite orders, where chi1 and X1 would be 0/0); where W = 0 (k = 0, or [k]_c . v_gal = 0)
    the coefficients are the standard ones, the paper's W -> 0 limit (``coefficients``).
    A W that is zero up to the rounding of the sines in [k]_c (|W dt| < 1e-12, e.g. at the
    Nyquist index, where [k]_c vanishes exactly) counts as zero.  Where 0 < |W dt| < 0.05 the
    closed forms lose about log10(1 / |W dt|) digits to the cancellation behind
    1 / (theta* - theta); there the same formulas are evaluated in 40-digit arithmetic
    (mpmath) from the float64 [k]_s, W.
    Returns complex arrays TC = theta^2 C, TS = theta^2 S/w_s, X1, X2, TX3 = theta^2 X3, X4."""
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    kcx, kcy, kcz = np.broadcast_arrays(*kc)
    std = coefficients(ks, dt)
    ws = C_LIGHT * np.sqrt(ksx ** 2 + ksy ** 2 + ksz ** 2)
    W = v_gal[0] * kcx + v_gal[1] * kcy + v_gal[2] * kcz
    gal = np.abs(W * dt) >= 1e-12
    Wg = np.where(gal, W, 0.5)     # placeholders away from every singularity where not used
    wsg = np.where(gal, ws, 1.0)   # W != 0 implies k != 0, so w_s > |W| > 0 there
    C, S_over_w = std["C"], std["S_over_w"]
    theta = np.exp(0.5j * Wg * dt)
    thetac = np.conj(theta)
    one_minus_C_over_w2 = np.where(gal, 2.0 * np.sin(0.5 * wsg * dt) ** 2 / wsg ** 2, 0.0)
    X1 = theta * (thetac - theta * C + 1j * Wg * theta * S_over_w) / (EPS0 * (wsg ** 2 - Wg ** 2))
    X2 = C_LIGHT ** 2 / (thetac - theta) * (thetac * X1 - theta * one_minus_C_over_w2 / EPS0)
    X3 = C_LIGHT ** 2 / (thetac - theta) * (thetac * X1 - thetac * one_minus_C_over_w2 / EPS0)
    X4 = 1j * Wg * X1 - theta ** 2 * S_over_w / EPS0
    th2 = theta ** 2
    out = {"TC": np.where(gal, th2 * C, C + 0j), "TS": np.where(gal, th2 * S_over_w, S_over_w + 0j),
           "X1": np.where(gal, X1, std["X1"] + 0j), "X2": np.where(gal, X2, std["X2"] + 0j),
           "TX3": np.where(gal, th2 * X3, std["X3"] + 0j), "X4": np.where(gal, X4, std["X4"] + 0j)}
    for idx in zip(*np.nonzero(gal & (np.abs(W * dt) < 0.05))):
        vals = _galilean_mp(float(ksx[idx]), float(ksy[idx]), float(ksz[idx]), float(W[idx]), dt)
        for key, val in vals.items():
            out[key][idx] = val
    return out


def _galilean_mp(kx, ky, kz, W, dt):
    """The closed forms of ``galilean_coefficients`` for one mode in 40-digit arithmetic."""
    import mpmath as mp
    with mp.workdps(40):
        c2, eps0 = mp.mpf(C_LIGHT) ** 2, mp.mpf(EPS0)
        ws = mp.sqrt(c2 * (mp.mpf(kx) ** 2 + mp.mpf(ky) ** 2 + mp.mpf(kz) ** 2))
        W, dt = mp.mpf(W), mp.mpf(dt)
        C, S = mp.cos(ws * dt), mp.sin(ws * dt)
        theta = mp.expj(W * dt / 2)
        thetac = mp.conj(theta)
        omc = (1 - C) / ws ** 2
        X1 = theta * (thetac - theta * C + 1j * W * theta * S / ws) / (eps0 * (ws ** 2 - W ** 2))
        X2 = c2 / (thetac - theta) * (thetac * X1 - theta * omc / eps0)
        X3 = c2 / (thetac - theta) * (thetac * X1 - thetac * omc / eps0)
        X4 = 1j * W * X1 - theta ** 2 * S / ws / eps0
        th2 = theta ** 2
        vals = {"TC": th2 * C, "TS": th2 * S / ws, "X1": X1, "X2": X2, "TX3": th2 * X3, "X4": X4}
        return {k: complex(v) for k, v in vals.items()}


def update_galilean(Eh, Bh, Jh, rho_old_h, rho_new_h, ks, gc):
    """One standard-Galilean-PSATD step of the paper-convention spectra (Sec. 4.3):
      B' = theta^2 C B - i theta^2 (S/w_s) [k]_s x E + i X1 [k]_s x J
      E' = theta^2 C E + i c^2 theta^2 (S/w_s) [k]_s x B + X4 J + i (theta^2 X3 rho^n - X2 rho^{n+1}) [k]_s"""
    kxE = cross(ks, Eh)
    kxB = cross(ks, Bh)
    kxJ = cross(ks, Jh)
    TC, TS, X1, X2, TX3, X4 = gc["TC"], gc["TS"], gc["X1"], gc["X2"], gc["TX3"], gc["X4"]
    B_new = tuple(TC * Bh[d] - 1j * TS * kxE[d] + 1j * X1 * kxJ[d] for d in range(3))
    E_new = tuple(TC * Eh[d] + 1j * C_LIGHT ** 2 * TS * kxB[d] + X4 * Jh[d]
                  + 1j * (TX3 * rho_old_h - X2 * rho_new_h) * ks[d] for d in range(3))
    return E_new, B_new


# ---------------------------------------------------------------- averaged Galilean PSATD (Sec. 4.4)

def _averaged_closed(ws, W, dt, m):
    """Psi1, Psi2, Y1, Y2, Y3, Y4 of Sec. 4.4 for one mode (or arrays), with the math module ``m``
    (numpy or mpmath) providing cos, sin, exp; c = eps0 = 1 as everywhere in the oracle:
      Psi1 = (theta^3 (w S3 + i W C3) - theta (w S1 + i W C1)) / ((w^2 - W^2) dt)
      Psi2 = (theta^3 (C3 - i W S3 / w) - theta (C1 - i W S1 / w)) / ((w^2 - W^2) dt)
      Psi3 = -i theta (theta^2 - 1) / (W dt)
      Y1 = (1 - Psi1 - i W Psi2) / (eps0 (w^2 - W^2))
      Y2 = i c^2 (eps0 w^2 Y1 - Psi3 + Psi1) / (eps0 w^2 (theta^2 - 1))
      Y3 = i c^2 (Psi3 - Psi1 - eps0 theta^2 w^2 Y1) / (eps0 w^2 (theta^2 - 1))
      Y4 = i W Y1 + Psi2 / eps0
    with C_m = cos(m w dt / 2), S_m = sin(m w dt / 2)."""
    c2, eps0 = C_LIGHT ** 2, EPS0
    C1, S1 = m.cos(ws * dt / 2), m.sin(ws * dt / 2)
    C3, S3 = m.cos(3 * ws * dt / 2), m.sin(3 * ws * dt / 2)
    th = m.exp(1j * W * dt / 2)
    th2, th3 = th * th, th * th * th
    den = (ws * ws - W * W) * dt
    Psi1 = (th3 * (ws * S3 + 1j * W * C3) - th * (ws * S1 + 1j * W * C1)) / den
    Psi2 = (th3 * (C3 - 1j * W * S3 / ws) - th * (C1 - 1j * W * S1 / ws)) / den
    Psi3 = -1j * th * (th2 - 1) / (W * dt)
    Y1 = (1 - Psi1 - 1j * W * Psi2) / (eps0 * (ws * ws - W * W))
    Y2 = 1j * c2 * (eps0 * ws * ws * Y1 - Psi3 + Psi1) / (eps0 * ws * ws * (th2 - 1))
    Y3 = 1j * c2 * (Psi3 - Psi1 - eps0 * th2 * ws * ws * Y1) / (eps0 * ws * ws * (th2 - 1))
    Y4 = 1j * W * Y1 + Psi2 / eps0
    return {"Psi1": Psi1, "Psi2": Psi2, "Y1": Y1, "Y2": Y2, "Y3": Y3, "Y4": Y4}


def averaged_coefficients(ks, kc, v_gal, dt):
    """Per-mode coefficients of the averaged Galilean update (Sec. 4.4, eqs.
    ``eq_update_B/E_with_rho_averaged``).  Reading (the paper defers the averaging to its
    reference): <f>^{n+1} is the mean of the step's exact solution, continued with the same
    J^{n+1/2}, over [t_n + dt/2, t_n + 3 dt/2] -- the interval whose end points give the
    theta, C1, S1, theta^3, C3, S3 of Psi1 and Psi2.
    The closed forms cancel across the whole spectrum (Y2, Y3 twice: through Y1 and through
    theta^2 - 1; float64 leaves ~1e-13) and have removable singularities at W = 0 (Psi3, Y2, Y3)
    and at w_s = W (k = 0 on grids, |v_gal| < c), so every mode is evaluated in 40-digit
    arithmetic (mpmath), at W = 1e-15 w_s where W = 0 and at w_s = 1e-12 where w_s = 0 (80 digits
    there): the coefficients are smooth functions of (w_s^2, W), so these values equal the limits
    to ~1e-15 relative."""
    import mpmath as mp
    ksx, ksy, ksz = np.broadcast_arrays(*ks)
    kcx, kcy, kcz = np.broadcast_arrays(*kc)
    ws = C_LIGHT * np.sqrt(ksx ** 2 + ksy ** 2 + ksz ** 2)
    W = v_gal[0] * kcx + v_gal[1] * kcy + v_gal[2] * kcz
    W = np.where(np.abs(W * dt) < 1e-12, 0.0, W)
    out = {k: np.zeros(ws.shape, dtype=complex) for k in ("Psi1", "Psi2", "Y1", "Y2", "Y3", "Y4")}
    for idx in np.ndindex(*ws.shape):
        w, Wv = float(ws[idx]), float(W[idx])
        with mp.workdps(80 if (w == 0 or Wv == 0) else 40):
            wm = mp.mpf(w) if w != 0 else mp.mpf("1e-12")
            Wm = mp.mpf(Wv) if Wv != 0 else wm * mp.mpf("1e-15")
            vals = _averaged_closed(wm, Wm, mp.mpf(dt), mp)
            for key, val in vals.items():
                out[key][idx] = complex(val)
    return out


def update_averaged(Eh, Bh, Jh, rho_old_h, rho_new_h, ks, ac):
    """The averaged fields of Sec. 4.4 from the step's start values:
      <B>^{n+1} = Psi1 B^n + i Psi2 [k]_s x E^n + i Y1 [k]_s x J^{n+1/2}
      <E>^{n+1} = Psi1 E^n - i c^2 Psi2 [k]_s x B^n + Y4 J^{n+1/2} + (Y3 rho^n + Y2 rho^{n+1}) [k]_s"""
    kxE = cross(ks, Eh)
    kxB = cross(ks, Bh)
    kxJ = cross(ks, Jh)
    P1, P2, Y1, Y2, Y3, Y4 = ac["Psi1"], ac["Psi2"], ac["Y1"], ac["Y2"], ac["Y3"], ac["Y4"]
    B_avg = tuple(P1 * Bh[d] + 1j * P2 * kxE[d] + 1j * Y1 * kxJ[d] for d in range(3))
    E_avg = tuple(P1 * Eh[d] - 1j * C_LIGHT ** 2 * P2 * kxB[d] + Y4 * Jh[d]
                  + (Y3 * rho_old_h + Y2 * rho_new_h) * ks[d] for d in range(3))
    return E_avg, B_avg


# ---------------------------------------------------------------- spectral current correction

def _has_direction(k2):
    """Modes whose modified wave vector is nonzero.  The centered [k]_c vanishes at the Nyquist index
    of an even axis in exact arithmetic; its sines leave ~1e-16 there, so a squared length below
    1e-24 of the largest counts as zero (the smallest genuine |[k]|^2 on grids of <= 1024 points
    is ~1e-5 of the largest)."""
    return k2 > 1e-24 * np.max(k2)


def current_correction(Jh, rho_old_h, rho_new_h, ks, dt):
    """Projection of the current onto the discrete continuity equation (reading of the charge
    conservation that Sec. 6 defers; the continuity law is the Fourier-space one of App. A,
    (rho^{n+1} - rho^n)/dt + i [k]_s . J = 0, with the same [k]_s as the field solver):
        J' = J - [k]_s ([k]_s . J - i (rho^{n+1} - rho^n)/dt) / |[k]_s|^2.
    J' - J is parallel to [k]_s (a discrete gradient), so [k]_s x J, and with it the B update
    and the transverse current, is unchanged.  Modes with |[k]_s| = 0 (k = 0; the Nyquist planes
    of the centered [k]_c) have no longitudinal direction and keep J.  Paper-convention spectra
    in and out."""
    kx, ky, kz = np.broadcast_arrays(*ks)
    k2 = kx * kx + ky * ky + kz * kz
    has = _has_direction(k2)
    k2s = np.where(has, k2, 1.0)
    mismatch = kx * Jh[0] + ky * Jh[1] + kz * Jh[2] - 1j * (rho_new_h - rho_old_h) / dt
    f = np.where(has, mismatch / k2s, 0.0)
    return (Jh[0] - kx * f, Jh[1] - ky * f, Jh[2] - kz * f)


def current_correction_transpose(gJ, g_old, g_new, ks, dt):
    """Conjugate transpose of ``current_correction``: the projection J -> J - [k]_s ([k]_s . J)/|k|^2
    is real symmetric, and J' depends on rho^{n+1} through + i [k]_s rho^{n+1} / (dt |k|^2) (and on
    rho^n with the opposite sign), which contribute conj(i / (dt |k|^2)) [k]_s . lambda.  Given the
    adjoint ``gJ`` of the corrected current, returns the adjoints of J, rho^n and rho^{n+1} with
    ``g_old``, ``g_new`` (those of the update itself) added."""
    kx, ky, kz = np.broadcast_arrays(*ks)
    k2 = kx * kx + ky * ky + kz * kz
    has = _has_direction(k2)
    s = np.where(has, (kx * gJ[0] + ky * gJ[1] + kz * gJ[2]) / np.where(has, k2, 1.0), 0.0)
    return ((gJ[0] - kx * s, gJ[1] - ky * s, gJ[2] - kz * s),
            g_old + 1j * s / dt, g_new - 1j * s / dt)
