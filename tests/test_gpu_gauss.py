"""Gauss's-law residual on the GPU (pic_gauss_residual) against the oracle's spectral residual:
random fields over several shapes (the half-spectrum weights of the kz = 0 and Nyquist planes
carry a different share of the sum on each), staggered and nodal solvers, finite and infinite order; and
fields that satisfy the order-2 Yee Gauss law exactly, where the residual is a rounding-level
number."""

import numpy as np
import pytest

from gpu_common import banner, put, rounded

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
