"""The fully staggered comparison cycle (PIC_STAGGERED_CYCLE) on the GPU against the oracle's:
every component gathered from and J deposited to its own Yee positions, no centering."""

import numpy as np
import pytest

from gpu_common import banner, max_rel, np64, oracle_species, periodic_pos_err, put, rounded

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import step as ostep  # noqa: E402
from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_order", [1, 3])
@pytest.mark.parametrize("v_gal", [(0.0, 0.0, 0.0), (0.0, 0.0, -0.9)])
def test_staggered_cycle_parity(dtype, shape_order, v_gal):
    shape = (16, 12, 24)
    banner(f"pic_step staggered cycle dtype={dtype} shape_order={shape_order} v_gal={v_gal}")
    wl = inputs.small(shape, ppc=2, shape_order=shape_order, center_order=8, dtype=dtype, u_th=0.1,
                      field_amp=0.05, seed=59)
    ctx = piclib.Context.for_workload(wl, flags=piclib.PIC_STAGGERED_CYCLE, v_gal=v_gal)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order, v_gal=v_gal,
                     staggered=True)
    osp = oracle_species(el, shape, wl.spacing)
    oion = oracle_species(ions, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oion], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    tol = 1e-10 if dtype == "f64" else 1e-4
    for n in range(3):
        piclib.pic_step(ctx.ctx, f, [el], 1)
        piclib.pic_sync(ctx.ctx)
        out = ostep.step(state, [osp], p, rho_static)
        for d in range(3):
            assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, (n, "E", d)
            assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, (n, "B", d)
            assert max_rel(np64(f.J_stag[d]), out["J_stag"][d]) <= tol, (n, "J", d)
        assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
        # the particles keep their order
        assert periodic_pos_err(el.positions(shape, wl.spacing), osp["pos"], p.lengths) <= (
            1e-11 if dtype == "f64" else 2e-5)
        u = np.stack([np64(x) for x in el.u], axis=1)
        assert np.max(np.abs(u - osp["u"])) <= (1e-11 if dtype == "f64" else 2e-5)
    ctx.close()
