"""Reverse mode of one hybrid PIC step (oracle).

Test infrastructure only (see ``oracle/__init__``).

One step (``step.step``, Sec. 2 cycle) maps the state (E^n, B^n on the Yee grid, rho^n,
positions x^n, momenta u^{n-1/2}) to the state at n+1.  ``step_vjp`` returns, for the
adjoint lambda of the state at n+1, the adjoint at n, by the chain rule through the
stages of the cycle in reverse order:
  field solve (Sec. 4.2)        -> conjugate transpose of the per-mode update
                                   (``push_fields_vjp``; brute force: ``push_fields_transpose``)
  centering (Sec. 3)            -> nodal-to-staggered and staggered-to-nodal are each
                                   other's transposes (same coefficients)
  deposition, gather            -> sums over the same shape stencils with the shape and its
                                   derivative (``deposit_vjp``, ``gather_vjp``)
  Boris rotation, v = u/gamma   -> Jacobians by complex-step differentiation of the forward
                                   functions themselves (``jacobian_vjp``)
Positions are absolute (physical units), as in ``particles``; their adjoints too.
"""

import numpy as np

from . import centering, particles, psatd, transforms
from .step import center_fields_s2n, push_fields
from .transforms import B_NAMES, E_NAMES, J_NAMES, OFFSETS


def push_fields_transpose(lam_E, lam_B, p):
    """dL/d(E, B, J, rho_old, rho_new) for dL/dE' = lam_E, dL/dB' = lam_B (lists of 3 arrays),
    by brute force: column c of the Jacobian is the response to the unit input c, and lambda
    contracts it to one gradient entry.  Obviously correct and slow (tiny grids).

    Returns a list of 11 arrays: E (3), B (3), J (3), rho_old, rho_new."""
    shape = p.shape
    grads = [np.zeros(shape) for _ in range(11)]
    for a in range(11):
        for idx in np.ndindex(*shape):
            x = [np.zeros(shape) for _ in range(11)]
            x[a][idx] = 1.0
            E, B = push_fields(x[0:3], x[3:6], x[6:9], x[9], x[10], p)
            grads[a][idx] = sum(float(np.sum(lam_E[d] * E[d]) + np.sum(lam_B[d] * B[d])) for d in range(3))
    return grads


def push_fields_vjp(lam_E, lam_B, p):
    """The same 11 arrays as ``push_fields_transpose``, from the conjugate-transposed update.

    The field solve is x -> Re IFFT(e^{+ik.d_a} M_ab e^{-ik.d_b} FFT x_b) per output a and input b
    (d the components' offsets); with numpy's unnormalised FFT its transpose is
    lambda_a -> Re IFFT(e^{+ik.d_b} conj(M_ab) e^{-ik.d_a} FFT lambda_a)."""
    if p.nodal:
        ks = psatd.centered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = {name: (0.0, 0.0, 0.0) for name in OFFSETS}
    else:
        ks = psatd.staggered_wave_vector(p.shape, p.spacing, p.psatd_order)
        offsets = OFFSETS
    coef = psatd.coefficients(ks, p.dt)
    lEh = [transforms.forward(lam_E[d], p.spacing, offsets[E_NAMES[d]]) for d in range(3)]
    lBh = [transforms.forward(lam_B[d], p.spacing, offsets[B_NAMES[d]]) for d in range(3)]
    gE, gB, gJ, g_old, g_new = psatd.update_transpose(lEh, lBh, ks, coef)
    if p.current_correction:
        gJ, g_old, g_new = psatd.current_correction_transpose(gJ, g_old, g_new, ks, p.dt)
    inv = lambda g, name: transforms.inverse(g, p.spacing, offsets[name])
    return ([inv(gE[d], E_NAMES[d]) for d in range(3)] + [inv(gB[d], B_NAMES[d]) for d in range(3)]
            + [inv(gJ[d], J_NAMES[d]) for d in range(3)] + [inv(g_old, "rho"), inv(g_new, "rho")])


def _axis_nodes_grad(xc, order):
    """[(node index, weight, d weight / d xc)] along one axis for positions ``xc`` in cells."""
    i0 = np.floor(xc).astype(np.int64)
    offsets = (0, 1) if order == 1 else (-1, 0, 1, 2)
    return [(i0 + o, particles.shape_1d(order, xc - (i0 + o)), particles.shape_1d_deriv(order, xc - (i0 + o)))
            for o in offsets]


def _stencil_grad(pos, shape, spacing, order):
    """Yield (linear node index, weight, gradient of the weight w.r.t. the position (3 arrays))."""
    nx, ny, nz = shape
    ax = _axis_nodes_grad(pos[:, 0] / spacing[0], order)
    ay = _axis_nodes_grad(pos[:, 1] / spacing[1], order)
    az = _axis_nodes_grad(pos[:, 2] / spacing[2], order)
    for ix, wx, gx in ax:
        for iy, wy, gy in ay:
            for iz, wz, gz in az:
                lin = (np.mod(ix, nx) * ny + np.mod(iy, ny)) * nz + np.mod(iz, nz)
                grad = (gx * wy * wz / spacing[0], wx * gy * wz / spacing[1], wx * wy * gz / spacing[2])
                yield lin, wx * wy * wz, grad


def gather_vjp(fields, pos, lam, spacing, order):
    """Adjoint of ``particles.gather`` (out[c, p] = sum_i S(x_p - x_i) F_c[i]) for dL/dout = lam.

    Returns (dL/dF_c arrays, dL/dpos of shape (Np, 3))."""
    shape = fields[0].shape
    n = int(np.prod(shape))
    flat = [np.asarray(f, dtype=np.float64).ravel() for f in fields]
    gF = [np.zeros(n) for _ in fields]
    gpos = np.zeros((pos.shape[0], 3))
    for lin, w, grad in _stencil_grad(pos, shape, spacing, order):
        for c, f in enumerate(flat):
            gF[c] += np.bincount(lin, weights=w * lam[c], minlength=n)
            for a in range(3):
                gpos[:, a] += grad[a] * lam[c] * f[lin]
    return [g.reshape(shape) for g in gF], gpos


def deposit_vjp(values, pos, lam_grids, shape, spacing, order):
    """Adjoint of ``particles.deposit`` (out_c[i] = sum_p values_c[p] S(x_p - x_i) / dV).

    Returns (dL/dvalues of shape (C, Np), dL/dpos of shape (Np, 3))."""
    dV = spacing[0] * spacing[1] * spacing[2]
    flat = [np.asarray(g, dtype=np.float64).ravel() for g in lam_grids]
    gval = np.zeros((len(values), pos.shape[0]))
    gpos = np.zeros((pos.shape[0], 3))
    for lin, w, grad in _stencil_grad(pos, shape, spacing, order):
        for c, (v, g) in enumerate(zip(values, flat)):
            gval[c] += w * g[lin] / dV
            for a in range(3):
                gpos[:, a] += grad[a] * v * g[lin] / dV
    return gval, gpos


def jacobian_vjp(fn, args, lam, h=1e-30):
    """lam^T (d fn / d arg) for every argument (arrays of shape (3, Np), one Jacobian per
    particle) by complex-step differentiation: the derivative along x_k is Im fn(x + i h e_k) / h,
    exact to rounding for a function analytic in its inputs (no subtraction, so no cancellation)."""
    out = []
    for ai, a in enumerate(args):
        g = np.zeros_like(np.asarray(a, dtype=np.float64))
        for k in range(g.shape[0]):
            pert = [np.asarray(x, dtype=np.complex128).copy() for x in args]
            pert[ai][k] += 1j * h
            col = np.imag(fn(*pert)) / h
            g[k] = np.sum(lam * col, axis=0)
        out.append(g)
    return out


def _velocity(u):
    return u / particles.gamma(u)


def _s2n_transpose(names, grads, p):
    """Transpose of the staggered-to-nodal centering (the nodal-to-staggered one)."""
    if p.nodal:
        return [np.array(g) for g in grads]
    m = p.center_order // 2
    return [centering.n2s(names[d], grads[d], m) for d in range(3)]


def _n2s_transpose(names, grads, p):
    if p.nodal:
        return [np.array(g) for g in grads]
    m = p.center_order // 2
    return [centering.s2n(names[d], grads[d], m) for d in range(3)]


def step_vjp(state, species, lam, p):
    """Adjoint of ``step.step`` at the state before the step.

    state: E_stag, B_stag (rho_old is not needed: the step is linear in it).
    species: list of dicts (pos, u, w, q, m) at time n.
    lam: dict E (3 arrays), B (3), rho (the adjoint of rho^{n+1}, the next step's rho_old),
    species: list of dicts pos (Np, 3), u (Np, 3), the adjoints of x^{n+1}, u^{n+1/2}.
    Returns the same structure for (E^n, B^n, rho^n, x^n, u^{n-1/2})."""
    if any(v != 0 for v in p.v_gal):
        raise NotImplementedError("the reverse mode covers the standard PSATD cycle (v_gal = 0)")
    E_nod, B_nod = center_fields_s2n(state["E_stag"], state["B_stag"], p)
    g = push_fields_vjp(lam["E"], lam["B"], p)
    gE, gB, gJs, g_rho_old, g_rho_new = g[0:3], g[3:6], g[6:9], g[9], g[10] + lam["rho"]
    gJ_nod = _n2s_transpose(J_NAMES, gJs, p)
    gEB_nod = [np.zeros(p.shape) for _ in range(6)]
    out_species = []
    for sp, ls in zip(species, lam["species"]):
        pos, u, qw = sp["pos"], sp["u"], sp["q"] * sp["w"]
        g_pos_new = np.array(ls["pos"], dtype=np.float64)
        g_u_new = np.array(ls["u"], dtype=np.float64).T
        if not np.isfinite(sp["m"]):  # immobile: rho from the unchanged positions only
            _, gpn = deposit_vjp([qw], pos, [g_rho_new], p.shape, p.spacing, p.shape_order)
            out_species.append({"pos": g_pos_new + gpn, "u": g_u_new.T})
            continue
        EB = particles.gather(list(E_nod) + list(B_nod), pos, p.spacing, p.shape_order)
        boris = lambda uu, E, B: particles.boris(uu, E, B, sp["q"], sp["m"], p.dt)
        u_new = boris(u.T, EB[:3], EB[3:])
        v = _velocity(u_new)
        pos_new = particles.wrap(pos + p.dt * v.T, p.lengths)
        pos_half = particles.wrap(pos + 0.5 * p.dt * v.T, p.lengths)
        # rho^{n+1} at x^{n+1}; J^{n+1/2} = q w v S(x^{n+1/2}) with x^{n+1/2} = x^n + dt v / 2
        gval, gph = deposit_vjp([qw * v[0], qw * v[1], qw * v[2]], pos_half, gJ_nod, p.shape, p.spacing,
                                p.shape_order)
        _, gpn = deposit_vjp([qw], pos_new, [g_rho_new], p.shape, p.spacing, p.shape_order)
        g_pos_new = g_pos_new + gpn
        gv = qw * gval + 0.5 * p.dt * gph.T + p.dt * g_pos_new.T
        g_pos = g_pos_new + gph
        g_u_new = g_u_new + jacobian_vjp(_velocity, [u_new], gv)[0]
        g_u, g_E, g_B = jacobian_vjp(boris, [u.T, EB[:3], EB[3:]], g_u_new)
        gF, gpg = gather_vjp(list(E_nod) + list(B_nod), pos, np.vstack([g_E, g_B]), p.spacing, p.shape_order)
        for c in range(6):
            gEB_nod[c] += gF[c]
        out_species.append({"pos": g_pos + gpg, "u": g_u.T})
    gE_s = _s2n_transpose(E_NAMES, gEB_nod[:3], p)
    gB_s = _s2n_transpose(B_NAMES, gEB_nod[3:], p)
    return {"E": [gE[d] + gE_s[d] for d in range(3)], "B": [gB[d] + gB_s[d] for d in range(3)],
            "rho": g_rho_old, "species": out_species}
