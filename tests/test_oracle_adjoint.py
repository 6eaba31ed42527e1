"""The oracle's reverse mode of the field solve, pinned by the paper's time reversal of the
vacuum update (App. B): with no sources the update is a rotation per mode, so its
transpose is the update with -dt.  CPU only."""

import numpy as np

from oracle import adjoint
from oracle.step import Params, push_fields


def test_vacuum_transpose_is_time_reversed_update():
    rng = np.random.default_rng(5)
    shape = (8, 8, 8)
    p = Params(shape, (1.0, 1.0, 1.0), 0.7, 1, 8, 16)
    lam_E = [rng.standard_normal(shape) for _ in range(3)]
    lam_B = [rng.standard_normal(shape) for _ in range(3)]
    g = adjoint.push_fields_transpose(lam_E, lam_B, p)
    zero = np.zeros(shape)
    p_back = Params(shape, (1.0, 1.0, 1.0), -0.7, 1, 8, 16)
    E_back, B_back = push_fields(lam_E, lam_B, [zero, zero, zero], zero, zero, p_back)
    for d in range(3):
        np.testing.assert_allclose(g[d], E_back[d], atol=1e-12)
        np.testing.assert_allclose(g[3 + d], B_back[d], atol=1e-12)


def test_transpose_satisfies_the_dot_product_identity():
    rng = np.random.default_rng(6)
    shape = (8, 8, 8)
    p = Params(shape, (1.0, 1.0, 1.0), 0.5, 3, 8, 16)
    lam_E = [rng.standard_normal(shape) for _ in range(3)]
    lam_B = [rng.standard_normal(shape) for _ in range(3)]
    x = [rng.standard_normal(shape) for _ in range(11)]
    g = adjoint.push_fields_transpose(lam_E, lam_B, p)
    E, B = push_fields(x[0:3], x[3:6], x[6:9], x[9], x[10], p)
    lhs = sum(np.sum(lam_E[d] * E[d]) + np.sum(lam_B[d] * B[d]) for d in range(3))
    rhs = sum(np.sum(g[a] * x[a]) for a in range(11))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)


# ---------------------------------------------------------------- reverse mode of the whole step

import pytest

from oracle import particles
from oracle.step import step


@pytest.mark.parametrize("nodal,correction", [(False, False), (True, False), (False, True), (True, True)])
def test_conjugate_transposed_update_matches_brute_force(nodal, correction):
    rng = np.random.default_rng(11)
    shape = (8, 8, 6)
    p = Params(shape, (1.0, 1.0, 1.0), 0.5, 1, 4, 8, nodal=nodal, current_correction=correction)
    lam_E = [rng.standard_normal(shape) for _ in range(3)]
    lam_B = [rng.standard_normal(shape) for _ in range(3)]
    brute = adjoint.push_fields_transpose(lam_E, lam_B, p)
    fast = adjoint.push_fields_vjp(lam_E, lam_B, p)
    for a in range(11):
        np.testing.assert_allclose(fast[a], brute[a], atol=1e-12)


@pytest.mark.parametrize("order", [1, 3])
def test_shape_derivative_matches_central_differences(order):
    rng = np.random.default_rng(12)
    d = rng.uniform(-2.2, 2.2, 2000)
    knots = np.array([-2.0, -1.0, 0.0, 1.0, 2.0])
    d = d[np.min(np.abs(d[:, None] - knots[None, :]), axis=1) > 1e-3]
    h = 1e-6
    fd = (particles.shape_1d(order, d + h) - particles.shape_1d(order, d - h)) / (2 * h)
    np.testing.assert_allclose(particles.shape_1d_deriv(order, d), fd, atol=1e-8)


def _random_particles(rng, shape, n):
    pos = rng.uniform(0.0, 1.0, (n, 3)) * np.asarray(shape, dtype=np.float64)[None, :]
    return pos


@pytest.mark.parametrize("order", [1, 3])
def test_gather_and_deposit_adjoints_against_directional_differences(order):
    rng = np.random.default_rng(13)
    shape, spacing = (8, 6, 8), (1.0, 1.5, 0.75)
    pos = _random_particles(rng, shape, 40) * np.asarray(spacing)[None, :]
    F = [rng.standard_normal(shape) for _ in range(2)]
    lam = rng.standard_normal((2, 40))
    dF = [rng.standard_normal(shape) for _ in range(2)]
    dpos = rng.standard_normal((40, 3))
    h = 1e-6
    Lg = lambda s: np.sum(lam * particles.gather([F[c] + s * dF[c] for c in range(2)], pos + s * dpos, spacing,
                                                 order))
    gF, gpos = adjoint.gather_vjp(F, pos, lam, spacing, order)
    fd = (Lg(h) - Lg(-h)) / (2 * h)
    an = sum(np.sum(gF[c] * dF[c]) for c in range(2)) + np.sum(gpos * dpos)
    assert abs(fd - an) <= 1e-6 * (abs(an) + 1)
    vals = rng.standard_normal((2, 40))
    dvals = rng.standard_normal((2, 40))
    lamg = [rng.standard_normal(shape) for _ in range(2)]
    Ld = lambda s: sum(np.sum(lamg[c] * o) for c, o in enumerate(
        particles.deposit([vals[c] + s * dvals[c] for c in range(2)], pos + s * dpos, shape, spacing, order)))
    gval, gpos = adjoint.deposit_vjp(list(vals), pos, lamg, shape, spacing, order)
    fd = (Ld(h) - Ld(-h)) / (2 * h)
    an = np.sum(gval * dvals) + np.sum(gpos * dpos)
    assert abs(fd - an) <= 1e-6 * (abs(an) + 1)


def test_boris_adjoint_closed_form_without_magnetic_field():
    # B = 0: u^{n+1/2} = u^{n-1/2} + (q dt / m) E, so lambda passes to u unchanged and to E times q dt / m
    rng = np.random.default_rng(14)
    u, E, lam = (rng.standard_normal((3, 30)) for _ in range(3))
    q, m, dt = -1.0, 1.0, 0.5
    fn = lambda uu, EE, BB: particles.boris(uu, EE, BB, q, m, dt)
    gu, gE, gB = adjoint.jacobian_vjp(fn, [u, E, np.zeros((3, 30))], lam)
    np.testing.assert_allclose(gu, lam, atol=1e-14)
    np.testing.assert_allclose(gE, (q * dt / m) * lam, atol=1e-14)


def test_boris_adjoint_against_central_differences():
    rng = np.random.default_rng(15)
    u, E, B, lam = (rng.standard_normal((3, 30)) for _ in range(4))
    du, dE, dB = (rng.standard_normal((3, 30)) for _ in range(3))
    fn = lambda uu, EE, BB: particles.boris(uu, EE, BB, -1.0, 1.0, 0.5)
    h = 1e-6
    L = lambda s: np.sum(lam * fn(u + s * du, E + s * dE, B + s * dB))
    gu, gE, gB = adjoint.jacobian_vjp(fn, [u, E, B], lam)
    fd = (L(h) - L(-h)) / (2 * h)
    an = np.sum(gu * du) + np.sum(gE * dE) + np.sum(gB * dB)
    assert abs(fd - an) <= 1e-7 * (abs(an) + 1)


def _state_dot(lam, st, sps, lengths):
    """<lambda, state> with positions entering as they are (the caller differences them)."""
    s = sum(np.sum(lam["E"][d] * st["E_stag"][d]) + np.sum(lam["B"][d] * st["B_stag"][d]) for d in range(3))
    s += np.sum(lam["rho"] * st["rho_old"])
    for ls, sp in zip(lam["species"], sps):
        s += np.sum(ls["u"] * sp["u"])
    return s


@pytest.mark.parametrize("order,nodal,immobile,correction", [(1, False, False, False), (3, False, True, False),
                                                              (3, True, False, False), (3, False, True, True)])
def test_step_adjoint_against_directional_differences(order, nodal, immobile, correction):
    """<vjp(lambda), delta> = d/ds <lambda, step(x + s delta)> at s = 0 (central differences, FP64)."""
    rng = np.random.default_rng(16 + order)
    shape, spacing = (8, 8, 6), (1.0, 1.0, 1.0)
    p = Params(shape, spacing, 0.5, order, 4, 8, nodal=nodal, current_correction=correction)
    n = 48
    state = {"E_stag": [0.3 * rng.standard_normal(shape) for _ in range(3)],
             "B_stag": [0.3 * rng.standard_normal(shape) for _ in range(3)],
             "rho_old": 0.1 * rng.standard_normal(shape)}
    sps = [{"pos": _random_particles(rng, shape, n), "u": 0.3 * rng.standard_normal((n, 3)),
            "w": rng.uniform(0.5, 1.5, n), "q": -1.0, "m": 1.0}]
    if immobile:
        sps.append({"pos": _random_particles(rng, shape, 16), "u": np.zeros((16, 3)), "w": np.ones(16),
                    "q": 1.0, "m": np.inf})
    lam = {"E": [rng.standard_normal(shape) for _ in range(3)], "B": [rng.standard_normal(shape) for _ in range(3)],
           "rho": rng.standard_normal(shape),
           "species": [{"pos": rng.standard_normal((s["pos"].shape[0], 3)),
                        "u": rng.standard_normal((s["pos"].shape[0], 3))} for s in sps]}
    delta = {"E": [rng.standard_normal(shape) for _ in range(3)], "B": [rng.standard_normal(shape) for _ in range(3)],
             "rho": rng.standard_normal(shape),
             "species": [{"pos": rng.standard_normal((s["pos"].shape[0], 3)),
                          "u": rng.standard_normal((s["pos"].shape[0], 3)) * np.isfinite(s["m"])} for s in sps]}

    def run(s):
        st = {"E_stag": [state["E_stag"][d] + s * delta["E"][d] for d in range(3)],
              "B_stag": [state["B_stag"][d] + s * delta["B"][d] for d in range(3)],
              "rho_old": state["rho_old"] + s * delta["rho"]}
        sp = [dict(sp0, pos=sp0["pos"] + s * ds["pos"], u=sp0["u"] + s * ds["u"])
              for sp0, ds in zip(sps, delta["species"])]
        start = [x["pos"].copy() for x in sp]
        step(st, sp, p)
        return st, sp, start

    h = 1e-6
    st_p, sp_p, st0_p = run(h)
    st_m, sp_m, st0_m = run(-h)
    fd = (_state_dot(lam, st_p, sp_p, p.lengths) - _state_dot(lam, st_m, sp_m, p.lengths)) / (2 * h)
    L = np.asarray(p.lengths)[None, :]
    for ls, a, b in zip(lam["species"], sp_p, sp_m):  # positions: periodic difference
        dpos = a["pos"] - b["pos"]
        dpos -= L * np.round(dpos / L)
        fd += np.sum(ls["pos"] * dpos) / (2 * h)
    g = adjoint.step_vjp(state, [dict(s) for s in sps], lam, p)
    an = sum(np.sum(g["E"][d] * delta["E"][d]) + np.sum(g["B"][d] * delta["B"][d]) for d in range(3))
    an += np.sum(g["rho"] * delta["rho"])
    for gs, ds in zip(g["species"], delta["species"]):
        an += np.sum(gs["pos"] * ds["pos"]) + np.sum(gs["u"] * ds["u"])
    assert abs(fd - an) <= 2e-7 * (abs(an) + 1), (fd, an)
