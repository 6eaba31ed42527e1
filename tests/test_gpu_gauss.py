"""Gauss's-law residual on the GPU (pic_gauss_residual) against the oracle's spectral residual:
random fields over several shapes (the half-spectrum weights of the kz = 0 and Nyquist planes
carry a different share of the sum on each), staggered and nodal solvers, finite and infinite order; and
fields that satisfy the order-2 Yee Gauss law exactly, where the residual is a rounding-level
number."""

import numpy as np
import pytest

from gpu_common import banner, np64, put, rounded

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import diagnostics as odiag  # noqa: E402
from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402

SPACING = (0.8, 1.1, 0.9)


def _run(shape, dtype, order, nodal, E, rho):
    flags = piclib.PIC_NODAL_SOLVER if nodal else 0
    ctx = piclib.Context(shape, SPACING, 0.4, 1, 8, order, dtype, flags=flags)
    f = piclib.Fields(shape, dtype)
    put(f.E_stag, E)
    put([f.rho_old], [rho])
    got = piclib.pic_gauss_residual(ctx.ctx, f)
    ctx.close()
    return got


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 24, 18), (12, 8, 54), (32, 16, 64)])
@pytest.mark.parametrize("order,nodal", [(16, False), (0, False), (8, True)])
def test_gauss_residual_matches_oracle(dtype, shape, order, nodal):
    banner(f"pic_gauss_residual vs oracle dtype={dtype} shape={shape} order={order} nodal={nodal}")
    arrs = rounded(inputs.random_grid(shape, seed=51, count=4), dtype)
    E, rho = arrs[:3], arrs[3]
    got = _run(shape, dtype, order, nodal, E, rho)
    ref = odiag.gauss_residual(E, rho, SPACING, order, nodal=nodal)
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert abs(got - ref) <= tol * ref, (got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gauss_residual_of_a_gauss_satisfying_field(dtype):
    """rho := the order-2 Yee divergence of E: the residual is zero up to rounding."""
    shape = (16, 12, 24)
    banner(f"pic_gauss_residual of a Gauss-satisfying field dtype={dtype} shape={shape}")
    E = rounded(inputs.random_grid(shape, seed=52, count=3), dtype)
    rho = sum((E[d] - np.roll(E[d], 1, axis=d)) / SPACING[d] for d in range(3))
    got = _run(shape, dtype, 2, False, E, rho)
    ref = odiag.gauss_residual(E, rounded([rho], dtype)[0], SPACING, 2)
    # f32: rho rounded to the run precision leaves a relative residual of order eps
    assert got < (1e-13 if dtype == "f64" else 5e-6), (got, ref)


def test_gauss_residual_without_charge_and_bad_arguments():
    shape = (8, 8, 8)
    banner(f"pic_gauss_residual, zero rho and argument errors, shape={shape}")
    E = inputs.random_grid(shape, seed=53, count=3)
    got = _run(shape, "f64", 2, False, E, np.zeros(shape))
    ref = odiag.gauss_residual(E, np.zeros(shape), SPACING, 2)
    assert abs(got - ref) <= 1e-12 * ref
    ctx = piclib.Context(shape, SPACING, 0.4, 1, 8, 2, "f64")
    f = piclib.Fields(shape, "f64")
    f.rho_old = None
    with pytest.raises(RuntimeError, match="rho_old"):
        piclib.pic_gauss_residual(ctx.ctx, f)
    ctx.close()


def _run_continuity(shape, dtype, order, nodal, J, r0, r1, dt=0.4):
    flags = piclib.PIC_NODAL_SOLVER if nodal else 0
    ctx = piclib.Context(shape, SPACING, dt, 1, 8, order, dtype, flags=flags)
    f = piclib.Fields(shape, dtype)
    put(f.J_nod if nodal else f.J_stag, J)
    put([f.rho_old, f.rho_new], [r0, r1])
    got = piclib.pic_continuity_residual(ctx.ctx, f)
    ctx.close()
    return got


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 24, 18), (32, 16, 64)])
@pytest.mark.parametrize("order,nodal", [(16, False), (0, False), (8, True)])
def test_continuity_residual_matches_oracle(dtype, shape, order, nodal):
    banner(f"pic_continuity_residual vs oracle dtype={dtype} shape={shape} order={order} nodal={nodal}")
    arrs = rounded(inputs.random_grid(shape, seed=54, count=5), dtype)
    J, r0, r1 = arrs[:3], arrs[3], arrs[4]
    got = _run_continuity(shape, dtype, order, nodal, J, r0, r1)
    ref = odiag.continuity_residual(J, r0, r1, SPACING, 0.4, order, nodal=nodal)
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert abs(got - ref) <= tol * ref, (got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_continuity_residual_of_a_charge_conserving_pair(dtype):
    """rho^{n+1} := rho^n - dt (order-2 Yee divergence of J): the residual is zero up to rounding."""
    shape, dt = (16, 12, 24), 0.4
    banner(f"pic_continuity_residual of a charge-conserving pair dtype={dtype} shape={shape}")
    arrs = rounded(inputs.random_grid(shape, seed=55, count=4), dtype)
    J, r0 = arrs[:3], arrs[3]
    r1 = r0 - dt * sum((J[d] - np.roll(J[d], 1, axis=d)) / SPACING[d] for d in range(3))
    got = _run_continuity(shape, dtype, 2, False, J, r0, r1, dt)
    assert got < (1e-12 if dtype == "f64" else 5e-5), got


def test_continuity_residual_after_a_step():
    """One hybrid step of a small cubic workload in FP64: the residual of its deposited sources
    (rho^n saved before the step, rho^{n+1} and J^{n+1/2} after it) against the oracle's on the same
    arrays; direct deposition leaves it well above rounding."""
    shape = (16, 12, 24)
    banner(f"pic_continuity_residual after one pic_step, FP64, shape={shape}")
    wl = inputs.small(shape, ppc=2, shape_order=3, center_order=8, dtype="f64", u_th=0.1, field_amp=0.02, seed=7)
    ctx = piclib.Context.for_workload(wl)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, "f64")
    ions = piclib.Species.from_host(wl.ions, shape, "f64")
    ctx.init_charge(f, el, ions)
    rho_n = f.rho_old.clone()
    piclib.pic_step(ctx.ctx, f, [el], 1)
    piclib.pic_sync(ctx.ctx)
    rho_n1 = f.rho_old.clone()
    f.rho_new.copy_(rho_n1)
    f.rho_old.copy_(rho_n)
    got = piclib.pic_continuity_residual(ctx.ctx, f)
    ref = odiag.continuity_residual([np64(x) for x in f.J_stag], np64(rho_n), np64(rho_n1), wl.spacing, wl.dt,
                                    wl.psatd_order)
    ctx.close()
    assert abs(got - ref) <= 1e-10 * ref, (got, ref)
    assert got > 1e-6
