"""PIC_DETERMINISTIC on the GPU: the same step from the same state gives bitwise the same fields and
particles whatever the order of the particles in memory (fixed-point deposition with
order-independent tile scales; particles kept in the caller's order)."""

import numpy as np
import pytest

from gpu_common import banner, np64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402


def _run(wl, order_perm, dtype, flags, nsteps):
    import copy
    w2 = copy.deepcopy(wl)
    for name in ("cell", "off", "u", "w"):
        setattr(w2.electrons, name, getattr(w2.electrons, name)[order_perm])
    ctx = piclib.Context.for_workload(w2, flags=flags)
    f = ctx.fields_from_workload(w2)
    el = piclib.Species.from_host(w2.electrons, wl.shape, dtype)
    ions = piclib.Species.from_host(w2.ions, wl.shape, dtype)
    ctx.init_charge(f, el, ions)
    piclib.pic_step(ctx.ctx, f, [el], nsteps)
    piclib.pic_sync(ctx.ctx)
    out = {"E": [np64(t) for t in f.E_stag], "B": [np64(t) for t in f.B_stag], "rho": np64(f.rho_old),
           "J": [np64(t) for t in f.J_nod]}
    inv = np.argsort(order_perm)
    out["cell"] = el.cell.cpu().numpy()[inv]
    out["off"] = [np64(t)[inv] for t in el.off]
    out["u"] = [np64(t)[inv] for t in el.u]
    ctx.close()
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("order,extra", [(1, 0), (3, 0), (3, piclib.PIC_CURRENT_CORRECTION)])
def test_deterministic_step_is_bitwise_reproducible(dtype, order, extra):
    shape = (24, 16, 32)
    banner(f"PIC_DETERMINISTIC bitwise reproducibility dtype={dtype} order={order} extra_flags={extra}")
    wl = inputs.small(shape, ppc=4, shape_order=order, center_order=8, dtype=dtype, u_th=0.4, field_amp=0.05,
                      seed=91)
    rng = np.random.default_rng(92)
    ident = np.arange(wl.electrons.n)
    flags = piclib.PIC_DETERMINISTIC | extra
    a = _run(wl, ident, dtype, flags, 3)
    b = _run(wl, rng.permutation(wl.electrons.n), dtype, flags, 3)
    c = _run(wl, ident[::-1].copy(), dtype, flags, 3)
    for other in (b, c):
        for key in ("E", "B", "J", "off", "u"):
            for d in range(3):
                assert np.array_equal(a[key][d], other[key][d]), (key, d)
        assert np.array_equal(a["rho"], other["rho"])
        assert np.array_equal(a["cell"], other["cell"])
