"""One hybrid nodal-staggered PSATD PIC cycle (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 2, the hybrid cycle: push particles -> deposit rho, J on the nodal grid ->
centre J from the nodal to the Yee grid -> solve Maxwell's equations on the
Yee grid in Fourier space -> centre E, B from the Yee to the nodal grid ->
gather E, B from the nodal grid.  One call of ``step`` starts from the state
(E, B on the Yee grid at time n; positions x^n; momenta u^{n-1/2};
rho^n on the nodes) and runs, in this order:
  1. E_nod, B_nod = staggered-to-nodal centering of E^n, B^n;
  2. gather + Boris push: u^{n-1/2} -> u^{n+1/2}, x^n -> x^{n+1};
  3. deposit rho^{n+1} (plus a static background) and J^{n+1/2} on the nodes;
  4. J on the Yee grid = nodal-to-staggered centering of J;
  5. standard PSATD update of (E, B) in the paper's Fourier convention;
  6. back to real space; rho^n <- rho^{n+1}.
Immobile species (m = inf) are never pushed and deposit rho only.

With a nonzero ``Params.v_gal`` the field solve is the standard Galilean PSATD update
(Sec. 4.3) and the particles move in the Galilean frame, x += dt (v - v_gal) (the frame
whose Fourier-space Maxwell equations carry the -v_gal . grad term of Sec. 4.3).

With ``Params.averaged`` (Sec. 4.4) the state also carries the averaged fields E_avg, B_avg:
the particles are pushed by their centering, and each step replaces them by the means of the
step's solution over [t_n + dt/2, t_n + 3 dt/2] (``psatd.averaged_coefficients``) while E, B
advance with the Galilean update.

With ``Params.staggered`` it runs the fully staggered cycle the paper compares against (Sec. 2;
the staggered runs of Sec. 5.2-5.3): every field and J on the Yee grid, each component gathered
from and deposited to its own Yee positions (the shape centred on x_i + delta_c), rho on the
nodes, no centering, the same staggered PSATD update.

With ``Params.nodal`` the same function runs the standard nodal PSATD cycle the paper
compares against (Sec. 2, first cycle figure; Sec. 4.1 [k]_c): every field on the nodes,
no centering, the update with the centered modified wave numbers.

With ``Params.current_correction`` the field solve first projects J^{n+1/2} onto the
Fourier-space continuity equation of App. A (``psatd.current_correction``), so that the update,
which carries Gauss's law exactly when continuity holds, keeps it step after step (standard
PSATD only; Sec. 6 leaves charge conservation open, this is the reading used).
"""

from dataclasses import dataclass

import numpy as np

from . import centering, particles, psatd, transforms
from .transforms import B_NAMES, E_NAMES, J_NAMES, OFFSETS


@dataclass
class Params:
    shape: tuple            # (nx, ny, nz)
    spacing: tuple          # (dx, dy, dz)
    dt: float
    shape_order: int = 1    # 1 = CIC, 3 = cubic B-spline
    center_order: int = 8   # 2 m_c
    psatd_order: int = 16   # 2 m_p for [k]_s; 0 = infinite
    nodal: bool = False     # the nodal comparison cycle: every field on the nodes, [k]_c, no centering
    v_gal: tuple = (0.0, 0.0, 0.0)  # Galilean velocity (Sec. 4.3); zero = standard PSATD
    averaged: bool = False  # averaged Galilean PSATD (Sec. 4.4): particles see the averaged fields
    staggered: bool = False  # the fully staggered comparison cycle: Yee gather and deposition, no centering
    current_correction: bool = False  # project J onto the Fourier-space continuity equation before the solve

    @property
    def lengths(self):
        return tuple(n * d for n, d in zip(self.shape, self.spacing))


def _yee_shift(name, p):
    """The half-cell offset vector of a component's Yee position (physical units)."""
    return np.asarray(OFFSETS[name], dtype=np.float64) * np.asarray(p.spacing, dtype=np.float64)


def center_fields_s2n(E_stag, B_stag, p):
    if p.nodal or p.staggered:  # nodal cycle: the state is nodal; staggered cycle: gathered where it lives
        return [np.array(a) for a in E_stag], [np.array(a) for a in B_stag]
    m = p.center_order // 2
    E_nod = [centering.s2n(E_NAMES[d], E_stag[d], m) for d in range(3)]
    B_nod = [centering.s2n(B_NAMES[d], B_stag[d], m) for d in range(3)]
    return E_nod, B_nod


def center_current_n2s(J_nod, p):
    if p.nodal or p.staggered:  # staggered cycle: J was deposited on the Yee grid
        return [np.array(a) for a in J_nod]
    m = p.center_order // 2
    return [centering.n2s(J_NAMES[d], J_nod[d], m) for d in range(3)]


def gather_fields(E_nod, B_nod, pos, p):
    """E, B at the particles, shape (6, Np): from the nodes (one weight set), or in the staggered
    cycle each component from its own Yee positions, S(x_p - (x_i + delta_c))."""
    if p.staggered:
        return np.stack([particles.gather([F], pos - _yee_shift(name, p)[None, :], p.spacing, p.shape_order)[0]
                         for F, name in zip(list(E_nod) + list(B_nod), E_NAMES + B_NAMES)])
    return particles.gather(list(E_nod) + list(B_nod), pos, p.spacing, p.shape_order)


def gather_push(sp, E_nod, B_nod, p):
    """Advance one species in place; returns v^{n+1/2} (3, Np) and the half-step positions."""
    pos, u = sp["pos"], sp["u"]
    if not np.isfinite(sp["m"]):
        return np.zeros((3, pos.shape[0])), pos.copy()
    EB = gather_fields(E_nod, B_nod, pos, p)
    u_new = particles.boris(u.T, EB[:3], EB[3:], sp["q"], sp["m"], p.dt)
    v = u_new / particles.gamma(u_new)
    # in the Galilean frame (coordinates moving with v_gal) a particle moves at v - v_gal
    w = v.T - np.asarray(p.v_gal, dtype=np.float64)[None, :]
    pos_half = particles.wrap(pos + 0.5 * p.dt * w, p.lengths)
    pos_new = particles.wrap(pos + p.dt * w, p.lengths)
    sp["pos"] = pos_new
    sp["u"] = u_new.T.copy()
    return v, pos_half


def deposit_rho(species, p, rho_static=None):
    rho = np.zeros(p.shape) if rho_static is None else np.array(rho_static, dtype=np.float64)
    for sp in species:
        rho += particles.deposit([sp["q"] * sp["w"]], sp["pos"], p.shape, p.spacing, p.shape_order)[0]
    return rho


def deposit_current(sp, v, pos_half, p):
    qw = sp["q"] * sp["w"]
    if p.staggered:  # J^d onto its own Yee positions
        return [particles.deposit([qw * v[d]], pos_half - _yee_shift(J_NAMES[d], p)[None, :], p.shape, p.spacing,
                                  p.shape_order)[0] for d in range(3)]
    return particles.deposit([qw * v[0], qw * v[1], qw * v[2]], pos_half, p.shape, p.spacing, p.shape_order)


def push_fields(E_stag, B_stag, J_stag, rho_old, rho_new, p):
    """Standard PSATD update of the Yee-grid fields from time n to n+1 (Sec. 4.2).

    Nodal cycle (p.nodal): the same equations with the centered [k]_c, every component
    transformed at the nodes (zero offsets)."""
    if p.nodal:
        ks = psatd.centered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = {name: (0.0, 0.0, 0.0) for name in OFFSETS}
    else:
        ks = psatd.staggered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = OFFSETS
    fw = lambda f, name: transforms.forward(f, p.spacing, offsets[name])
    Eh = [fw(E_stag[d], E_NAMES[d]) for d in range(3)]
    Bh = [fw(B_stag[d], B_NAMES[d]) for d in range(3)]
    Jh = [fw(J_stag[d], J_NAMES[d]) for d in range(3)]
    rho_old_h = fw(rho_old, "rho")
    rho_new_h = fw(rho_new, "rho")
    if p.current_correction:
        if any(v != 0 for v in p.v_gal) or p.averaged:
            raise ValueError("the current correction is stated for the standard PSATD continuity equation")
        if p.nodal and p.psatd_order == 0:
            raise ValueError("the nodal solver at infinite order has no real derivative at the Nyquist index")
        Jh = psatd.current_correction(Jh, rho_old_h, rho_new_h, ks, p.dt)
    if any(v != 0 for v in p.v_gal):  # standard Galilean PSATD (Sec. 4.3)
        kc = psatd.centered_wave_vector(p.shape, p.spacing, p.psatd_order)
        gc = psatd.galilean_coefficients(ks, kc, p.v_gal, p.dt)
        E_new, B_new = psatd.update_galilean(Eh, Bh, Jh, rho_old_h, rho_new_h, ks, gc)
    else:
        E_new, B_new = psatd.update(Eh, Bh, Jh, rho_old_h, rho_new_h, ks, psatd.coefficients(ks, p.dt))
    E_out = [transforms.inverse(E_new[d], p.spacing, offsets[E_NAMES[d]]) for d in range(3)]
    B_out = [transforms.inverse(B_new[d], p.spacing, offsets[B_NAMES[d]]) for d in range(3)]
    return E_out, B_out


_AVERAGED_CACHE = {}


def averaged_fields(E_stag, B_stag, J_stag, rho_old, rho_new, p):
    """<E>^{n+1}, <B>^{n+1} of the averaged Galilean update (Sec. 4.4) on the Yee grid, from the
    step's start fields and sources (the Galilean update itself advances E, B)."""
    if p.nodal:
        ks = psatd.centered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = {name: (0.0, 0.0, 0.0) for name in OFFSETS}
    else:
        ks = psatd.staggered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = OFFSETS
    key = (p.shape, p.spacing, p.psatd_order, p.dt, tuple(p.v_gal), p.nodal)
    if key not in _AVERAGED_CACHE:  # slow (arbitrary precision): once per configuration
        kc = psatd.centered_wave_vector(p.shape, p.spacing, p.psatd_order)
        _AVERAGED_CACHE[key] = psatd.averaged_coefficients(ks, kc, p.v_gal, p.dt)
    ac = _AVERAGED_CACHE[key]
    fw = lambda f, name: transforms.forward(f, p.spacing, offsets[name])
    E_avg, B_avg = psatd.update_averaged([fw(E_stag[d], E_NAMES[d]) for d in range(3)],
                                         [fw(B_stag[d], B_NAMES[d]) for d in range(3)],
                                         [fw(J_stag[d], J_NAMES[d]) for d in range(3)],
                                         fw(rho_old, "rho"), fw(rho_new, "rho"), ks, ac)
    return ([transforms.inverse(E_avg[d], p.spacing, offsets[E_NAMES[d]]) for d in range(3)],
            [transforms.inverse(B_avg[d], p.spacing, offsets[B_NAMES[d]]) for d in range(3)])


def step(state, species, p, rho_static=None):
    """Advance ``state`` (dict: E_stag, B_stag, rho_old) and ``species`` (list of dicts) by one cycle.

    Returns a dict of the intermediate arrays of the step (for stage-by-stage parity)."""
    if p.averaged:  # the particles see the averaged fields (state["E_avg"], ["B_avg"] at time n)
        E_nod, B_nod = center_fields_s2n(state["E_avg"], state["B_avg"], p)
    else:
        E_nod, B_nod = center_fields_s2n(state["E_stag"], state["B_stag"], p)
    J_nod = [np.zeros(p.shape) for _ in range(3)]
    for sp in species:
        v, pos_half = gather_push(sp, E_nod, B_nod, p)
        if np.isfinite(sp["m"]):
            Jc = deposit_current(sp, v, pos_half, p)
            for d in range(3):
                J_nod[d] += Jc[d]
    rho_new = deposit_rho(species, p, rho_static)
    J_stag = center_current_n2s(J_nod, p)
    if p.averaged:
        state["E_avg"], state["B_avg"] = averaged_fields(state["E_stag"], state["B_stag"], J_stag, state["rho_old"],
                                                         rho_new, p)
    E_out, B_out = push_fields(state["E_stag"], state["B_stag"], J_stag, state["rho_old"], rho_new, p)
    state["E_stag"], state["B_stag"], state["rho_old"] = E_out, B_out, rho_new
    return {"E_nod": E_nod, "B_nod": B_nod, "J_nod": J_nod, "J_stag": J_stag, "rho_new": rho_new}
