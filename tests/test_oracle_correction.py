"""Pins of the oracle's spectral current correction (``psatd.current_correction``).

The paper leaves charge conservation to future work (Sec. 6); the reading used projects
J^{n+1/2} onto the Fourier-space continuity equation of App. A with the solver's own [k]_s.
What the mathematics fixes, checked here against real-space finite differences written out
with textbook stencils (not the oracle's spectral operators):
* the corrected current satisfies the order-2 and order-4 staggered continuity equations
  exactly (the order-2m [k]_s is the symbol of those stencils);
* the change is a discrete gradient: its staggered curl vanishes;
* a current that already satisfies continuity is left unchanged;
* a full hybrid step with the correction keeps Gauss's law, which the direct deposition alone
  does not.
"""

import numpy as np
import pytest

from oracle import diagnostics, psatd, transforms
from oracle.step import Params, deposit_rho, step
from oracle.transforms import J_NAMES, OFFSETS

SHAPE, SPACING, DT = (8, 10, 6), (0.7, 1.1, 0.9), 0.37

# textbook staggered first-derivative weights over +-h/2, +-3h/2
STENCIL = {2: [(1.0, 0)], 4: [(9.0 / 8.0, 0), (-1.0 / 24.0, 1)]}


def _div_yee(J, order):
    """Divergence at the nodes of J on the Yee grid (J_d at +1/2 cell along d)."""
    out = np.zeros(J[0].shape)
    for d in range(3):
        for c, s in STENCIL[order]:
            out += c * (np.roll(J[d], -s, axis=d) - np.roll(J[d], s + 1, axis=d)) / SPACING[d]
    return out


def _diff_up(f, axis, order):
    """Derivative of a field living at integer positions along ``axis``, evaluated half a cell above."""
    out = np.zeros(f.shape)
    for c, s in STENCIL[order]:
        out += c * (np.roll(f, -(s + 1), axis=axis) - np.roll(f, s, axis=axis)) / SPACING[axis]
    return out


def _curl_yee(J, order):
    """Curl on the faces of an edge (E-like) Yee field: (d_y J_z - d_z J_y, ...)."""
    return [_diff_up(J[2], 1, order) - _diff_up(J[1], 2, order),
            _diff_up(J[0], 2, order) - _diff_up(J[2], 0, order),
            _diff_up(J[1], 0, order) - _diff_up(J[0], 1, order)]


def _correct(J, r0, r1, order, nodal=False):
    offs = {n: ((0.0, 0.0, 0.0) if nodal else OFFSETS[n]) for n in J_NAMES}
    ks = (psatd.centered_wave_vector if nodal else psatd.staggered_wave_vector)(SHAPE, SPACING, order)
    Jh = [transforms.forward(J[d], SPACING, offs[J_NAMES[d]]) for d in range(3)]
    r0h = transforms.forward(r0, SPACING, (0.0, 0.0, 0.0))
    r1h = transforms.forward(r1, SPACING, (0.0, 0.0, 0.0))
    Jc = psatd.current_correction(Jh, r0h, r1h, ks, DT)
    return [transforms.inverse(Jc[d], SPACING, offs[J_NAMES[d]]) for d in range(3)]


def _sources(seed):
    rng = np.random.default_rng(seed)
    J = [rng.standard_normal(SHAPE) for _ in range(3)]
    r0, r1 = rng.standard_normal(SHAPE), rng.standard_normal(SHAPE)
    r1 += np.mean(r0) - np.mean(r1)  # the k = 0 mode: total charge conserved
    return J, r0, r1


@pytest.mark.parametrize("order", [2, 4])
def test_corrected_current_satisfies_the_finite_difference_continuity_equation(order):
    J, r0, r1 = _sources(61)
    before = np.abs((r1 - r0) / DT + _div_yee(J, order)).max()
    Jc = _correct(J, r0, r1, order)
    after = np.abs((r1 - r0) / DT + _div_yee(Jc, order)).max()
    assert before > 1.0
    assert after < 1e-12 * before
    assert diagnostics.continuity_residual(Jc, r0, r1, SPACING, DT, order) < 1e-13


@pytest.mark.parametrize("order", [2, 4])
def test_correction_is_a_discrete_gradient(order):
    J, r0, r1 = _sources(62)
    dJ = [a - b for a, b in zip(_correct(J, r0, r1, order), J)]
    assert max(np.abs(c).max() for c in dJ) > 0.1
    for c in _curl_yee(dJ, order):
        assert np.abs(c).max() < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_correction_keeps_a_current_that_already_satisfies_continuity(order):
    J, r0, _ = _sources(63)
    r1 = r0 - DT * _div_yee(J, order)
    Jc = _correct(J, r0, r1, order)
    for a, b in zip(Jc, J):
        np.testing.assert_allclose(a, b, atol=1e-12)


def test_nodal_correction_satisfies_continuity_where_the_centered_derivative_exists():
    """Nodal solver, order 2: [k]_c is the symbol of (f(x+h) - f(x-h)) / (2h).  It vanishes on the
    Nyquist planes of the even axes, which keep their current, so the residual is checked with
    the mismatch on those planes projected out first."""
    J, r0, r1 = _sources(64)
    Jc = _correct(J, r0, r1, 2, nodal=True)
    res = (r1 - r0) / DT + sum((np.roll(Jc[d], -1, axis=d) - np.roll(Jc[d], 1, axis=d)) / (2 * SPACING[d])
                               for d in range(3))
    rh = np.fft.fftn(res)
    ny = np.zeros(SHAPE, dtype=bool)
    for a, n in enumerate(SHAPE):
        idx = [slice(None)] * 3
        idx[a] = n // 2
        ny[tuple(idx)] = True
    assert np.abs(rh[~ny]).max() < 1e-11 * np.abs(np.fft.fftn((r1 - r0) / DT)).max()


def _plasma_state(correction):
    from paper_2106_12919_amd import inputs
    wl = inputs.small((8, 8, 12), ppc=2, shape_order=3, center_order=4, field_amp=0.0, u_th=0.2)
    p = Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order,
               current_correction=correction)
    el = {"pos": wl.electrons.positions(wl.spacing), "u": wl.electrons.u.copy(), "w": wl.electrons.w,
          "q": wl.electrons.q, "m": wl.electrons.m}
    ions = {"pos": wl.ions.positions(wl.spacing), "u": wl.ions.u, "w": wl.ions.w, "q": 1.0, "m": np.inf}
    rho_static = deposit_rho([ions], p)
    zero = [np.zeros(wl.shape) for _ in range(3)]
    state = {"E_stag": [z.copy() for z in zero], "B_stag": [z.copy() for z in zero],
             "rho_old": deposit_rho([el], p, rho_static)}
    return p, el, rho_static, state


def test_step_with_correction_keeps_gauss_law():
    """E = B = 0 with neutralising ions is Gauss-consistent; the update carries Gauss's law exactly
    when continuity holds (Sec. 4.2 / App. A), so with the correction the residual stays at rounding
    level every step, while the direct deposition alone leaves an O(1) relative residual."""
    for correction, lo, hi in ((True, 0.0, 1e-11), (False, 1e-3, np.inf)):
        p, el, rho_static, state = _plasma_state(correction)
        for _ in range(3):
            step(state, [el], p, rho_static)
            g = diagnostics.gauss_residual(state["E_stag"], state["rho_old"], p.spacing, p.psatd_order)
            assert lo <= g <= hi, (correction, g)


def test_correction_leaves_the_magnetic_update_unchanged():
    """J' - J is longitudinal, so one step from the same state gives the same B either way."""
    outs = []
    for correction in (False, True):
        p, el, rho_static, state = _plasma_state(correction)
        step(state, [el], p, rho_static)
        outs.append(state)
    for d in range(3):
        np.testing.assert_allclose(outs[1]["B_stag"][d], outs[0]["B_stag"][d], atol=1e-14)
    assert max(np.abs(outs[1]["E_stag"][d] - outs[0]["E_stag"][d]).max() for d in range(3)) > 1e-6
