"""Stage-by-stage parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case feeds both sides the same seeded inputs (rounded to the run precision
first, so the comparison isolates the kernels' arithmetic).  Tolerances:
FP64 cases use a few hundred ulps of the output scale; FP32 cases use bounds
derived from the operation count of each stage (see the per-test comments).
"""

import numpy as np
import pytest

from gpu_common import EPS, banner, max_rel, np64, oracle_species, periodic_pos_err, put, rounded

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import centering as ocent  # noqa: E402
from oracle import fornberg  # noqa: E402
from oracle import step as ostep  # noqa: E402
from oracle.transforms import B_NAMES, E_NAMES, J_NAMES  # noqa: E402
from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402

TD = {"f32": torch.float32, "f64": torch.float64}


def centering_tol(dtype, m, scale):
    # sum of 2m products with coefficients alpha/2: error <= (2m+1) eps sum|alpha| max|in|
    a = sum(abs(float(x)) for x in fornberg.alpha_staggered(m))
    return (2 * m + 1) * EPS[dtype] * a * scale * 2


# every centering order on every shape whose smallest axis admits it (pic_init rejects an order
# above the smallest axis; tests/test_library_abi.py checks that rejection)
_CENTER_CASES = [(shape, order) for shape in [(16, 24, 32), (48, 16, 8), (32, 36, 64)]
                 for order in [2, 4, 8, 16, 32] if order <= min(shape)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,order", _CENTER_CASES)
def test_center_parity(dtype, order, shape):
    banner(f"center dtype={dtype} order={order} shape={shape}")
    m = order // 2
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), 0.5, 1, order, 16, dtype)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=100 + order, count=9), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_nod, src[6:9])
    piclib.pic_center(ctx.ctx, piclib.PIC_S2N, piclib.PIC_E, f)
    piclib.pic_center(ctx.ctx, piclib.PIC_S2N, piclib.PIC_B, f)
    piclib.pic_center(ctx.ctx, piclib.PIC_N2S, piclib.PIC_J, f)
    piclib.pic_sync(ctx.ctx)
    scale = max(np.max(np.abs(s)) for s in src)
    tol = centering_tol(dtype, m, scale) * (2 if dtype == "f32" else 4)
    for d in range(3):
        refE = ocent.s2n(E_NAMES[d], src[d], m)
        refB = ocent.s2n(B_NAMES[d], src[3 + d], m)
        refJ = ocent.n2s(J_NAMES[d], src[6 + d], m)
        # B is centred along two axes: the first pass's rounding is amplified by sum|alpha|
        a = sum(abs(float(x)) for x in fornberg.alpha_staggered(m))
        assert np.max(np.abs(np64(f.E_nod[d]) - refE)) <= tol
        assert np.max(np.abs(np64(f.B_nod[d]) - refB)) <= tol * (1 + a)
        assert np.max(np.abs(np64(f.J_stag[d]) - refJ)) <= tol
    ctx.close()


def fft_tol(dtype, shape):
    # forward + inverse real 3D FFTs (3 passes each), the update in between: the
    # componentwise error of a radix-2/4/8 FFT is bounded by ~ log2(N) eps times the
    # RMS scale (Higham, Accuracy and Stability, ch. 24); allow a factor 10 margin
    # on the max-norm and the 11-term update.
    n = np.prod(shape)
    return 10 * 2 * np.log2(n) * EPS[dtype] * 3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 24, 32), (12, 8, 48), (8, 8, 8), (24, 96, 16)])
@pytest.mark.parametrize("psatd_order", [16, 0])
def test_psatd_push_fields_parity(dtype, shape, psatd_order):
    banner(f"psatd_push_fields dtype={dtype} shape={shape} order={psatd_order}")
    dt = 0.5
    p = ostep.Params(shape, (1.0, 1.0, 1.0), dt, 1, 8, psatd_order)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), dt, 1, 8, psatd_order, dtype)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=7, count=11), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_stag, src[6:9])
    put([f.rho_old, f.rho_new], src[9:11])
    piclib.psatd_push_fields(ctx.ctx, f)
    piclib.pic_sync(ctx.ctx)
    E_ref, B_ref = ostep.push_fields(src[0:3], src[3:6], src[6:9], src[9], src[10], p)
    tol = fft_tol(dtype, shape)
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), E_ref[d]) <= tol, (d, max_rel(np64(f.E_stag[d]), E_ref[d]))
        assert max_rel(np64(f.B_stag[d]), B_ref[d]) <= tol, (d, max_rel(np64(f.B_stag[d]), B_ref[d]))
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 24, 32), (12, 8, 48)])
@pytest.mark.parametrize("psatd_order", [16, 0])
def test_psatd_push_fields_nodal_solver_parity(dtype, shape, psatd_order):
    """PIC_NODAL_SOLVER: the update with the centered [k]_c on nodal arrays."""
    banner(f"psatd_push_fields nodal solver dtype={dtype} shape={shape} order={psatd_order}")
    dt = 0.5
    p = ostep.Params(shape, (1.0, 1.0, 1.0), dt, 1, 8, psatd_order, nodal=True)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), dt, 1, 8, psatd_order, dtype, flags=piclib.PIC_NODAL_SOLVER)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=9, count=11), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_stag, src[6:9])
    put([f.rho_old, f.rho_new], src[9:11])
    piclib.psatd_push_fields(ctx.ctx, f)
    piclib.pic_sync(ctx.ctx)
    E_ref, B_ref = ostep.push_fields(src[0:3], src[3:6], src[6:9], src[9], src[10], p)
    tol = fft_tol(dtype, shape)
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), E_ref[d]) <= tol, (d, max_rel(np64(f.E_stag[d]), E_ref[d]))
        assert max_rel(np64(f.B_stag[d]), B_ref[d]) <= tol, (d, max_rel(np64(f.B_stag[d]), B_ref[d]))
    ctx.close()


def push_tols(dtype):
    # FP32: ~100 rounding steps on O(1)-conditioned quantities (64 gathered terms, Boris)
    return (1e-12, 1e-12) if dtype == "f64" else (3e-6, 3e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_order", [1, 3])
def test_gather_push_parity(dtype, shape_order):
    banner(f"gather_push dtype={dtype} shape_order={shape_order}")
    shape = (16, 24, 12)
    wl = inputs.small(shape, ppc=3, shape_order=shape_order, dtype=dtype, u_th=0.2, seed=21)
    ctx = piclib.Context.for_workload(wl)
    f = piclib.Fields(shape, dtype)
    nod = rounded(inputs.random_grid(shape, seed=22, count=6, amp=0.3), dtype)
    put(f.E_nod, nod[0:3])
    put(f.B_nod, nod[3:6])
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    osp = oracle_species(el, shape, wl.spacing)
    p = ostep.Params(shape, wl.spacing, wl.dt, shape_order, wl.center_order, wl.psatd_order)
    piclib.pic_gather_push(ctx.ctx, f, [el])
    piclib.pic_sync(ctx.ctx)
    ostep.gather_push(osp, nod[0:3], nod[3:6], p)
    tu, tx = push_tols(dtype)
    u_gpu = np.stack([np64(x) for x in el.u], axis=1)
    assert np.max(np.abs(u_gpu - osp["u"])) <= tu * (1 + np.max(np.abs(osp["u"])))
    assert periodic_pos_err(el.positions(shape, wl.spacing), osp["pos"], p.lengths) <= tx * 4
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_order", [1, 3])
def test_deposit_parity(dtype, shape_order):
    banner(f"deposit dtype={dtype} shape_order={shape_order}")
    shape = (16, 12, 24)
    wl = inputs.small(shape, ppc=4, shape_order=shape_order, dtype=dtype, u_th=0.3, seed=31)
    ctx = piclib.Context.for_workload(wl)
    f = piclib.Fields(shape, dtype)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    piclib.pic_deposit(ctx.ctx, [el, ions], f, piclib.PIC_DEP_RHO_AND_J)
    piclib.pic_sync(ctx.ctx)
    p = ostep.Params(shape, wl.spacing, wl.dt, shape_order, wl.center_order, wl.psatd_order)
    osp = oracle_species(el, shape, wl.spacing)
    oion = oracle_species(ions, shape, wl.spacing)
    rho_ref = ostep.deposit_rho([osp, oion], p)
    # the device takes x^{n+1/2} = x^{n+1} - dt v / 2 from the current (post-push) positions
    u = osp["u"].T
    from oracle import particles as opart
    v = u / opart.gamma(u)
    pos_half = opart.wrap(osp["pos"] - 0.5 * wl.dt * v.T, p.lengths)
    J_ref = ostep.deposit_current(osp, v, pos_half, p)
    # FP32: each node accumulates ~ppc * S^3 contributions in arbitrary (atomic) order
    tol = 1e-12 if dtype == "f64" else 64 * 4 * EPS["f32"] * 4
    assert max_rel(np64(f.rho_new), rho_ref) <= tol
    for d in range(3):
        assert max_rel(np64(f.J_nod[d]), J_ref[d]) <= tol
    # charge conservation of the deposit: electrons and ions cancel in total, to rounding
    # relative to the total electron charge
    qtot = float(torch.sum(f.rho_new.double()).item()) * np.prod(wl.spacing)
    qe = abs(float(np.sum(osp["q"] * osp["w"])))
    assert abs(qtot) <= (1e-13 if dtype == "f64" else 1e-6) * qe
    ctx.close()


def test_deposit_rho_only_and_static():
    banner("deposit rho-only with static background")
    shape = (8, 16, 12)
    wl = inputs.small(shape, ppc=2, shape_order=3, dtype="f64", seed=41)
    ctx = piclib.Context.for_workload(wl)
    f = piclib.Fields(shape, "f64")
    el = piclib.Species.from_host(wl.electrons, shape, "f64")
    ions = piclib.Species.from_host(wl.ions, shape, "f64")
    ctx.init_charge(f, el, ions)
    piclib.pic_sync(ctx.ctx)
    # electrons on top of their own ions: zero everywhere
    assert np.max(np.abs(np64(f.rho_old))) < 1e-15
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_order,shape,u_th,nsteps,flags", [
    (1, (16, 12, 24), 0.1, 3, 0), (3, (16, 12, 24), 0.1, 3, 0), (3, (8, 16, 24), 0.4, 4, 0),
    (1, (16, 12, 24), 0.1, 3, piclib.PIC_SPECTRAL_CENTERING), (3, (8, 16, 24), 0.4, 4, piclib.PIC_SPECTRAL_CENTERING),
    (1, (16, 12, 24), 0.1, 3, piclib.PIC_NODAL_SOLVER), (3, (8, 16, 24), 0.4, 3, piclib.PIC_NODAL_SOLVER)])
def test_step_parity_small(dtype, shape_order, shape, u_th, nsteps, flags):
    """Full hybrid cycles on small workloads: several deposition tiles, a radix-3 axis, partial
    tiles, axes of one and two tiles (periodic neighbours that coincide) and, with the hotter
    plasma, many particles changing tile between steps.  With PIC_SPECTRAL_CENTERING the
    centering is applied as its Fourier symbol and must still match the real-space oracle; with
    PIC_NODAL_SOLVER the nodal comparison cycle must match the oracle's nodal cycle."""
    banner(f"pic_step small dtype={dtype} shape_order={shape_order} shape={shape} u_th={u_th} flags={flags}")
    wl = inputs.small(shape, ppc=2, shape_order=shape_order, center_order=8, dtype=dtype, u_th=u_th,
                      field_amp=0.02, seed=51)
    # distinct weights double as particle identities (pic_step regroups particles by tile)
    wl.electrons.w = wl.electrons.w * (1.0 + 1e-3 * np.arange(wl.electrons.n) / wl.electrons.n)
    ctx = piclib.Context.for_workload(wl, flags=flags)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order,
                     nodal=bool(flags & piclib.PIC_NODAL_SOLVER))
    osp = oracle_species(el, shape, wl.spacing)
    oion = oracle_species(ions, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oion], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    tol = 1e-10 if dtype == "f64" else 1e-4
    for n in range(nsteps):
        piclib.pic_step(ctx.ctx, f, [el], 1)
        piclib.pic_sync(ctx.ctx)
        ostep.step(state, [osp], p, rho_static)
        for d in range(3):
            assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, (n, "E", d)
            assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, (n, "B", d)
        assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
        g_w = np64(el.w)
        gi, oi = np.argsort(g_w), np.argsort(osp["w"])
        assert np.array_equal(g_w[gi], osp["w"][oi] if dtype == "f64" else osp["w"][oi])
        g_pos = el.positions(shape, wl.spacing)[gi]
        g_u = np.stack([np64(x) for x in el.u], axis=1)[gi]
        assert periodic_pos_err(g_pos, osp["pos"][oi], p.lengths) <= (1e-11 if dtype == "f64" else 2e-5)
        assert np.max(np.abs(g_u - osp["u"][oi])) <= (1e-11 if dtype == "f64" else 2e-5)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_order", [1, 3])
def test_spectral_centering_multi_step(dtype, shape_order):
    """One pic_step call of several steps with PIC_SPECTRAL_CENTERING (nodal fields of the later
    steps come from the fused update) against the real-space oracle: the staggered state, rho,
    every particle, and the nodal fields of the final time level."""
    banner(f"pic_step spectral centering, 4 steps in one call, dtype={dtype} shape_order={shape_order}")
    shape, nsteps = (16, 12, 24), 4
    wl = inputs.small(shape, ppc=2, shape_order=shape_order, center_order=8, dtype=dtype, u_th=0.3,
                      field_amp=0.02, seed=53)
    wl.electrons.w = wl.electrons.w * (1.0 + 1e-3 * np.arange(wl.electrons.n) / wl.electrons.n)
    ctx = piclib.Context.for_workload(wl, flags=piclib.PIC_SPECTRAL_CENTERING)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    osp = oracle_species(el, shape, wl.spacing)
    oion = oracle_species(ions, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oion], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    piclib.pic_step(ctx.ctx, f, [el], nsteps)
    piclib.pic_sync(ctx.ctx)
    for _ in range(nsteps):
        out = ostep.step(state, [osp], p, rho_static)
    tol = 1e-10 if dtype == "f64" else 2e-4
    E_nod, B_nod = ostep.center_fields_s2n(state["E_stag"], state["B_stag"], p)
    J_stag = ostep.center_current_n2s(out["J_nod"], p)
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, ("E", d)
        assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, ("B", d)
        assert max_rel(np64(f.E_nod[d]), E_nod[d]) <= tol, ("E_nod", d)
        assert max_rel(np64(f.B_nod[d]), B_nod[d]) <= tol, ("B_nod", d)
        assert max_rel(np64(f.J_stag[d]), J_stag[d]) <= tol, ("J_stag", d)
    assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
    g_w = np64(el.w)
    gi, oi = np.argsort(g_w), np.argsort(osp["w"])
    g_pos = el.positions(shape, wl.spacing)[gi]
    g_u = np.stack([np64(x) for x in el.u], axis=1)[gi]
    assert periodic_pos_err(g_pos, osp["pos"][oi], p.lengths) <= (1e-11 if dtype == "f64" else 4e-5)
    assert np.max(np.abs(g_u - osp["u"][oi])) <= (1e-11 if dtype == "f64" else 4e-5)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_regroups_particles_by_tile(dtype):
    """After pic_step the particles are grouped by deposition tile and none is lost or duplicated."""
    banner(f"pic_step regroup dtype={dtype}")
    shape = (32, 16, 24)
    wl = inputs.small(shape, ppc=2, shape_order=3, center_order=4, dtype=dtype, u_th=0.2, seed=61)
    rng = np.random.default_rng(0)
    order = rng.permutation(wl.electrons.n)      # scramble the input order
    for name in ("cell", "off", "u", "w"):
        setattr(wl.electrons, name, getattr(wl.electrons, name)[order])
    wl.electrons.w = wl.electrons.w * (1.0 + 1e-3 * np.arange(wl.electrons.n) / wl.electrons.n)
    ctx = piclib.Context.for_workload(wl)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    w0 = np.sort(np64(el.w))
    piclib.pic_step(ctx.ctx, f, [el], 2)
    piclib.pic_sync(ctx.ctx)
    assert np.array_equal(np.sort(np64(el.w)), w0)
    ctx.close()
