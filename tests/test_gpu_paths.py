"""Parity with the oracle on the paths the timed and full-size runs take that the stage tests on
small grids do not reach: the 384- and 768-point FFT axes of the beam-driven-wake grid and every
axis length with transform kernels of its own, calls of several steps on grids whose transforms
carry the centering (every axis length has kernels of its own), one
pic_step call of several steps (E, B resident in Fourier space) for the standard, Galilean and
averaged Galilean cycles, grids of more tiles than the single-launch bucket scan and the LDS
bucket histogram hold, the beam-driven wake at 1/4 scale (gamma = 1000 beam), several species
in one call in every order (two mobile species; an immobile one first or between), calls without
particles (no species, or species of zero particles), grids with an axis of 1024 points, the
largest accepted, and species of one constant weight (no weight array)."""

import numpy as np
import pytest

from gpu_common import EPS, banner, max_rel, np64, oracle_species, periodic_pos_err, put, rounded

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import particles as opart  # noqa: E402
from oracle import step as ostep  # noqa: E402
from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402


def fft_tol(dtype, shape):
    # forward and inverse real 3D transforms around the 11-term update (as the stage tests)
    return 10 * 2 * np.log2(np.prod(shape)) * EPS[dtype] * 3


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(8, 384, 768), (384, 8, 24)])
def test_field_solve_on_the_beam_grid_axes(dtype, shape):
    """384- and 768-point axes: the z transform packs two real lines of 768 points; strided passes
    of 384 points along y (first shape) and x (second shape) use the narrow-tile layouts."""
    banner(f"psatd_push_fields on 384/768-point axes dtype={dtype} shape={shape}")
    dt = 0.5
    p = ostep.Params(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16, dtype)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=111, count=11), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_stag, src[6:9])
    put([f.rho_old, f.rho_new], src[9:11])
    piclib.psatd_push_fields(ctx.ctx, f)
    piclib.pic_sync(ctx.ctx)
    E_ref, B_ref = ostep.push_fields(src[0:3], src[3:6], src[6:9], src[9], src[10], p)
    tol = fft_tol(dtype, shape)
    for d in range(3):
        eE, eB = max_rel(np64(f.E_stag[d]), E_ref[d]), max_rel(np64(f.B_stag[d]), B_ref[d])
        assert eE <= tol and eB <= tol, (d, eE, eB, tol)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(64, 128, 256), (128, 64, 384), (256, 256, 64), (768, 12, 128), (8, 768, 24)])
def test_field_solve_on_the_specialised_axis_lengths(dtype, shape):
    """The transforms have kernels of their own for axes of 64, 128, 256, 384 and 768 points; these
    shapes put each of those lengths on x, y and z at least once (with a z pass whose last block holds
    fewer line pairs than the others: 128 x 64 lines in pairs of 5 at 384 points, FP32)."""
    banner(f"psatd_push_fields on specialised axis lengths dtype={dtype} shape={shape}")
    dt = 0.5
    p = ostep.Params(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16, dtype)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=112, count=11), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_stag, src[6:9])
    put([f.rho_old, f.rho_new], src[9:11])
    piclib.psatd_push_fields(ctx.ctx, f)
    piclib.pic_sync(ctx.ctx)
    E_ref, B_ref = ostep.push_fields(src[0:3], src[3:6], src[6:9], src[9], src[10], p)
    tol = fft_tol(dtype, shape)
    for d in range(3):
        eE, eB = max_rel(np64(f.E_stag[d]), E_ref[d]), max_rel(np64(f.B_stag[d]), B_ref[d])
        assert eE <= tol and eB <= tol, (d, eE, eB, tol)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(1024, 8, 16), (8, 1024, 16), (8, 16, 1024)])
def test_field_solve_at_the_largest_axis_length(dtype, shape):
    """Axes of 1024 points, the largest pic_init accepts, on x, y and z in turn: the generic
    transform kernels at their narrowest tiles (one or two lines per strided tile, one or two line
    pairs per z block)."""
    banner(f"psatd_push_fields on 1024-point axes dtype={dtype} shape={shape}")
    dt = 0.5
    p = ostep.Params(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), dt, 1, 8, 16, dtype)
    f = piclib.Fields(shape, dtype)
    src = rounded(inputs.random_grid(shape, seed=113, count=11), dtype)
    put(f.E_stag, src[0:3])
    put(f.B_stag, src[3:6])
    put(f.J_stag, src[6:9])
    put([f.rho_old, f.rho_new], src[9:11])
    piclib.psatd_push_fields(ctx.ctx, f)
    piclib.pic_sync(ctx.ctx)
    E_ref, B_ref = ostep.push_fields(src[0:3], src[3:6], src[6:9], src[9], src[10], p)
    tol = fft_tol(dtype, shape)
    for d in range(3):
        eE, eB = max_rel(np64(f.E_stag[d]), E_ref[d]), max_rel(np64(f.B_stag[d]), B_ref[d])
        assert eE <= tol and eB <= tol, (d, eE, eB, tol)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(16, 16, 1024), (16, 1024, 16)])
def test_step_at_the_largest_axis_length(dtype, shape):
    """One call of two full cycles on grids with a 1024-point axis (cubic shape, centering order
    16): the centering passes on 1024-point lines (in FP64 the fused x/y-then-z pass does not fit
    and separate passes run), 128 tiles along that axis, the generic transforms; every field and
    every particle against the oracle."""
    banner(f"pic_step on a grid with a 1024-point axis dtype={dtype} shape={shape}")
    wl = inputs.small(shape, ppc=1, shape_order=3, center_order=16, dtype=dtype, u_th=0.1, field_amp=0.05,
                      seed=142)
    _ids(wl)
    ctx = piclib.Context.for_workload(wl, flags=0)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    osp = oracle_species(el, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oracle_species(ions, shape, wl.spacing)], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    nsteps = 2
    piclib.pic_step(ctx.ctx, f, [el], nsteps)
    piclib.pic_sync(ctx.ctx)
    for _ in range(nsteps):
        out = ostep.step(state, [osp], p, rho_static)
    tol = 1e-10 if dtype == "f64" else 1e-4
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, ("E", d)
        assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, ("B", d)
        assert max_rel(np64(f.J_nod[d]), out["J_nod"][d]) <= tol, ("J", d)
    assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
    _compare_particles(el, osp, shape, wl.spacing, p.lengths, dtype, 1e-11 if dtype == "f64" else 2e-5,
                       1e-11 if dtype == "f64" else 2e-5)
    ctx.close()


@pytest.mark.parametrize("dtype,shape_order,center_order,variant", [
    ("f64", 3, 8, "standard"), ("f32", 3, 16, "standard"), ("f64", 1, 4, "standard"), ("f32", 1, 32, "standard"),
    ("f64", 3, 8, "galilean"), ("f64", 3, 8, "correction")])
def test_call_with_centering_in_the_transforms(dtype, shape_order, center_order, variant):
    """On a 64^3 grid every axis has transform kernels of its own, so a pic_step call of several
    steps runs the real-space centering inside the transforms on every step but the last (also with
    the Galilean solver and the current correction).  Against the oracle's real-space cycle: the
    final staggered state, the nodal fields of the last step's start, that step's J on the Yee grid,
    rho and every particle."""
    banner(f"pic_step with centering in the transforms, 4 steps dtype={dtype} shape={shape_order} "
           f"centering={center_order} variant={variant}")
    shape, nsteps = (64, 64, 64), 4
    v_gal = (0.0, 0.0, -0.9) if variant == "galilean" else (0.0, 0.0, 0.0)
    flags = piclib.PIC_CURRENT_CORRECTION if variant == "correction" else 0
    wl = inputs.small(shape, ppc=1, shape_order=shape_order, center_order=center_order, dtype=dtype, u_th=0.2,
                      field_amp=0.02, seed=71)
    _ids(wl)
    ctx = piclib.Context.for_workload(wl, flags=flags, v_gal=v_gal)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order, v_gal=v_gal,
                     current_correction=(variant == "correction"))
    osp = oracle_species(el, shape, wl.spacing)
    oion = oracle_species(ions, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oion], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    piclib.pic_step(ctx.ctx, f, [el], nsteps)
    piclib.pic_sync(ctx.ctx)
    for n in range(nsteps):
        if n == nsteps - 1:
            E_nod, B_nod = ostep.center_fields_s2n(state["E_stag"], state["B_stag"], p)
        out = ostep.step(state, [osp], p, rho_static)
    tol = 1e-10 if dtype == "f64" else 2e-4
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


def _ids(wl):
    """Distinct weights w0 2^-k-free (1 + p 2^-23), exact in FP32: particle identities."""
    base = 2.0 ** np.floor(np.log2(wl.electrons.w[0]))
    wl.electrons.w = base * (1.0 + np.arange(wl.electrons.n) * 2.0 ** -23)


def _compare_particles(el, osp, shape, spacing, lengths, dtype, tol_pos, tol_u):
    g_w = np64(el.w)
    gi, oi = np.argsort(g_w), np.argsort(osp["w"])
    assert np.array_equal(g_w[gi], osp["w"][oi])
    assert periodic_pos_err(el.positions(shape, spacing)[gi], osp["pos"][oi], lengths) <= tol_pos
    g_u = np.stack([np64(x) for x in el.u], axis=1)[gi]
    assert np.max(np.abs(g_u - osp["u"][oi])) <= tol_u


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("variant", ["standard", "galilean", "averaged"])
def test_one_call_of_four_steps(dtype, variant):
    """pic_step(..., 4): 7 forward transforms on entry, then 4 forward and 6 inverse per step with E, B
    kept in Fourier space, against four oracle steps (the bench's way of running the cycle)."""
    shape, nsteps = (16, 16, 24), 4
    v_gal = (0.0, 0.0, -0.9) if variant != "standard" else (0.0, 0.0, 0.0)
    flags = piclib.PIC_AVERAGED if variant == "averaged" else 0
    banner(f"pic_step 4 steps in one call dtype={dtype} variant={variant}")
    wl = inputs.small(shape, ppc=2, shape_order=3, center_order=8, dtype=dtype, u_th=0.2, field_amp=0.05, seed=113)
    _ids(wl)
    ctx = piclib.Context.for_workload(wl, flags=flags, v_gal=v_gal)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order, v_gal=v_gal,
                     averaged=(variant == "averaged"))
    osp = oracle_species(el, shape, wl.spacing)
    rho_static = ostep.deposit_rho([oracle_species(ions, shape, wl.spacing)], p)
    E0, B0 = rounded(wl.E, dtype), rounded(wl.B, dtype)
    state = {"E_stag": E0, "B_stag": B0, "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    if variant == "averaged":
        state["E_avg"], state["B_avg"] = [a.copy() for a in E0], [b.copy() for b in B0]
    piclib.pic_step(ctx.ctx, f, [el], nsteps)
    piclib.pic_sync(ctx.ctx)
    for _ in range(nsteps):
        ostep.step(state, [osp], p, rho_static)
    tol = 1e-10 if dtype == "f64" else 2e-4
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, ("E", d)
        assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, ("B", d)
        if variant == "averaged":
            assert max_rel(np64(f.E_avg[d]), state["E_avg"][d]) <= tol, ("<E>", d)
            assert max_rel(np64(f.B_avg[d]), state["B_avg"][d]) <= tol, ("<B>", d)
    assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
    _compare_particles(el, osp, shape, wl.spacing, p.lengths, dtype, 1e-11 if dtype == "f64" else 4e-5,
                       1e-11 if dtype == "f64" else 4e-5)
    ctx.close()


def _sparse_plasma(rng, shape, count, n0, u_th):
    """``count`` particles in distinct random cells, uniform offsets, Gaussian momenta."""
    nx, ny, nz = shape
    lin = rng.choice(nx * ny * nz, size=count, replace=False)
    cell = np.stack([lin // (ny * nz), (lin // nz) % ny, lin % nz], axis=1).astype(np.int64)
    return inputs.Species(cell=cell, off=rng.random((count, 3)), u=rng.normal(0.0, u_th, (count, 3)),
                          w=np.full(count, n0), q=-1.0, m=1.0)


@pytest.mark.parametrize("shape", [(32, 1024, 576), (16, 1024, 768)])
def test_deposit_and_gather_on_grids_of_many_tiles(shape):
    """36,864 and 24,576 tiles of 8^3 cells: more buckets than one scan launch (16,384) and, for the
    first, than the LDS histogram of the counting sort (32,768), so the three-launch scan and the
    global-histogram sort run.  FP32, CIC, one sparse particle per 16 cells; pic_deposit and
    pic_gather_push against the oracle's deposition and gather + push."""
    banner(f"deposit + gather_push on a grid of many tiles shape={shape}")
    dtype = "f32"
    rng = np.random.Generator(np.random.PCG64(121))
    n = int(np.prod(shape)) // 16
    sp = _sparse_plasma(rng, shape, n, 0.01, 0.2)
    sp.w = 0.01 * (1.0 + np.arange(n) * 2.0 ** -23)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), 0.5, 1, 8, 16, dtype)
    f = piclib.Fields(shape, dtype)
    el = piclib.Species.from_host(sp, shape, dtype)
    osp = oracle_species(el, shape, (1.0, 1.0, 1.0))
    p = ostep.Params(shape, (1.0, 1.0, 1.0), 0.5, 1, 8, 16)
    # deposition from the (rounded) positions, as pic_deposit after a push: J at x - dt v / 2
    piclib.pic_deposit(ctx.ctx, [el], f)
    piclib.pic_sync(ctx.ctx)
    rho_ref = ostep.deposit_rho([osp], p)
    u = osp["u"]
    v = (u / np.sqrt(1.0 + np.sum(u * u, axis=1))[:, None]).T
    pos_half = opart.wrap(osp["pos"] - 0.5 * p.dt * v.T, p.lengths)
    J_ref = ostep.deposit_current(osp, v, pos_half, p)
    tol = 1024 * EPS[dtype]
    assert max_rel(np64(f.rho_new), rho_ref) <= tol
    for d in range(3):
        assert max_rel(np64(f.J_nod[d]), J_ref[d]) <= tol, d
    # gather + push from random nodal fields
    fld = rounded(inputs.random_grid(shape, seed=122, count=6, amp=0.05), dtype)
    put(f.E_nod, fld[0:3])
    put(f.B_nod, fld[3:6])
    piclib.pic_gather_push(ctx.ctx, f, [el])
    piclib.pic_sync(ctx.ctx)
    ostep.gather_push(osp, fld[0:3], fld[3:6], p)
    # pic_gather_push keeps the caller's order
    assert periodic_pos_err(el.positions(shape, (1.0, 1.0, 1.0)), osp["pos"], p.lengths) <= 3e-6
    g_u = np.stack([np64(x) for x in el.u], axis=1)
    assert np.max(np.abs(g_u - osp["u"])) <= 3e-6
    ctx.close()


@pytest.mark.parametrize("flags", [0, piclib.PIC_KEEP_ORDER])
def test_beam96_one_step(flags):
    """The beam-driven wake at 1/4 scale (96 x 96 x 192, gamma = 1000 drive beam with its
    self-fields, 1 ppc plasma, cubic, centering 16), FP32, one step against the oracle: every field
    in the bench's launch configuration (particles regrouped by tile), and with PIC_KEEP_ORDER,
    where the particles stay in the caller's order, every particle as well."""
    banner(f"beam96 one step FP32 vs oracle flags={flags}")
    wl = inputs.config("beam96")
    dtype = "f32"
    ctx = piclib.Context.for_workload(wl, flags=flags)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, wl.shape, dtype)
    ions = piclib.Species.from_host(wl.ions, wl.shape, dtype)
    ctx.init_charge(f, el, ions)
    p = ostep.Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    osp = oracle_species(el, wl.shape, wl.spacing)
    rho_static = ostep.deposit_rho([oracle_species(ions, wl.shape, wl.spacing)], p)
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho([osp], p, rho_static)}
    piclib.pic_step(ctx.ctx, f, [el], 1)
    piclib.pic_sync(ctx.ctx)
    ostep.step(state, [osp], p, rho_static)
    tol = 1e-4
    # relative to the largest field component: the beam's B_z vanishes (rounding noise on both sides)
    scale = max(np.max(np.abs(a)) for a in state["E_stag"] + state["B_stag"])
    for d in range(3):
        assert np.max(np.abs(np64(f.E_stag[d]) - state["E_stag"][d])) <= tol * scale, ("E", d)
        assert np.max(np.abs(np64(f.B_stag[d]) - state["B_stag"][d])) <= tol * scale, ("B", d)
    assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
    if flags & piclib.PIC_KEEP_ORDER:
        assert periodic_pos_err(el.positions(wl.shape, wl.spacing), osp["pos"], p.lengths) <= 2e-5
        g_u = np.stack([np64(x) for x in el.u], axis=1)
        # the beam's u_z ~ 1000: relative to the largest momentum
        assert max_rel(g_u, osp["u"]) <= 2e-6
    ctx.close()


def _mobile(seed, q, m, shape, dtype):
    wl = inputs.small(shape, ppc=2, shape_order=3, center_order=8, dtype=dtype, u_th=0.25, field_amp=0.05,
                      seed=seed)
    _ids(wl)
    wl.electrons.q, wl.electrons.m = q, m
    return wl


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("order", ["ion,el,pos", "el,ion,pos", "el,pos"])
def test_several_species_in_one_call(dtype, order):
    """Species in one pic_step call: the first deposited one overwrites rho (from rho_static) and, if
    mobile, J; later ones add.  Electrons and positrons (two mobile species) with the ions either
    passed as an immobile species (first or between: rho accumulates while J is first written by
    the first mobile one) or as the static background."""
    shape = (16, 16, 24)
    banner(f"pic_step several species dtype={dtype} order={order}")
    a = _mobile(131, -1.0, 1.0, shape, dtype)
    b = _mobile(132, +1.0, 1.0, shape, dtype)
    ctx = piclib.Context.for_workload(a, flags=0)
    f = ctx.fields_from_workload(a)
    el = piclib.Species.from_host(a.electrons, shape, dtype)
    po = piclib.Species.from_host(b.electrons, shape, dtype)
    ion = piclib.Species.from_host(a.ions, shape, dtype)
    p = ostep.Params(shape, a.spacing, a.dt, a.shape_order, a.center_order, a.psatd_order)
    osp = {"el": oracle_species(el, shape, a.spacing), "pos": oracle_species(po, shape, a.spacing),
           "ion": oracle_species(ion, shape, a.spacing)}
    dev = {"el": el, "pos": po, "ion": ion}
    names = order.split(",")
    rho_static = None
    if "ion" not in names:  # the ions as the static background
        piclib.pic_deposit(ctx.ctx, [ion], f, piclib.PIC_DEP_RHO_ONLY)
        f.rho_static = f.rho_new.clone()
        rho_static = ostep.deposit_rho([osp["ion"]], p)
    piclib.pic_deposit(ctx.ctx, [dev[k] for k in names], f, piclib.PIC_DEP_RHO_ONLY)
    f.rho_old.copy_(f.rho_new)
    state = {"E_stag": rounded(a.E, dtype), "B_stag": rounded(a.B, dtype),
             "rho_old": ostep.deposit_rho([osp[k] for k in names], p, rho_static)}
    tol = 1e-10 if dtype == "f64" else 1e-4
    for n in range(3):
        piclib.pic_step(ctx.ctx, f, [dev[k] for k in names], 1)
        piclib.pic_sync(ctx.ctx)
        out = ostep.step(state, [osp[k] for k in names], p, rho_static)
        for d in range(3):
            assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, (n, "E", d)
            assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, (n, "B", d)
            assert max_rel(np64(f.J_nod[d]), out["J_nod"][d]) <= tol, (n, "J", d)
        assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
        for k in ("el", "pos"):
            _compare_particles(dev[k], osp[k], shape, a.spacing, p.lengths, dtype,
                               1e-11 if dtype == "f64" else 2e-5, 1e-11 if dtype == "f64" else 2e-5)
    # the immobile species did not move (pic_step may have regrouped it by tile)
    if "ion" in names:
        g, r = ion.positions(shape, a.spacing), osp["ion"]["pos"]
        g, r = g[np.lexsort(g.T[::-1])], r[np.lexsort(r.T[::-1])]
        assert np.array_equal(g, r)
    ctx.close()


def _no_particles(q, m, dtype):
    td = torch.float32 if dtype == "f32" else torch.float64
    z = [torch.zeros(0, dtype=td, device="cuda") for _ in range(7)]
    return piclib.Species(torch.zeros(0, dtype=torch.int32, device="cuda"), z[0:3], z[3:6], z[6], q, m)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape,species", [((16, 12, 24), "none"), ((64, 64, 128), "none"),
                                           ((64, 64, 128), "empty"), ((16, 16, 24), "empty,el,empty")])
def test_calls_without_particles(dtype, shape, species):
    """The source-free case: with no species, or only species of zero particles, one call of three
    steps is the vacuum field solve around the static charge (rho^{n+1} = rho_static, J = 0), on a
    grid with partial tiles (generic transforms, separate centering passes) and on one whose
    transforms carry the centering.  Species of zero particles around a mobile one change nothing:
    the mobile one still writes the sources first."""
    banner(f"pic_step without particles dtype={dtype} shape={shape} species={species}")
    wl = _mobile(141, -1.0, 1.0, shape, dtype)
    ctx = piclib.Context.for_workload(wl, flags=0)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, shape, dtype)
    ions = piclib.Species.from_host(wl.ions, shape, dtype)
    empty = _no_particles(-1.0, 1.0, dtype)
    names = [] if species == "none" else species.split(",")
    dev = [el if k == "el" else empty for k in names]
    # rho_static from the ions; rho_old from the species passed (rho_static alone without particles)
    ctx.init_charge(f, empty if "el" not in names else el, ions)
    p = ostep.Params(shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    rho_static = ostep.deposit_rho([oracle_species(ions, shape, wl.spacing)], p)
    osp = [oracle_species(el, shape, wl.spacing)] if "el" in names else []
    state = {"E_stag": rounded(wl.E, dtype), "B_stag": rounded(wl.B, dtype),
             "rho_old": ostep.deposit_rho(osp, p, rho_static)}
    nsteps = 3
    piclib.pic_step(ctx.ctx, f, dev, nsteps)
    piclib.pic_sync(ctx.ctx)
    for _ in range(nsteps):
        out = ostep.step(state, osp, p, rho_static)
    tol = 1e-10 if dtype == "f64" else 1e-4
    for d in range(3):
        assert max_rel(np64(f.E_stag[d]), state["E_stag"][d]) <= tol, ("E", d)
        assert max_rel(np64(f.B_stag[d]), state["B_stag"][d]) <= tol, ("B", d)
        if osp:
            assert max_rel(np64(f.J_nod[d]), out["J_nod"][d]) <= tol, ("J", d)
        else:
            assert not torch.any(f.J_nod[d] != 0), ("J", d)
    assert max_rel(np64(f.rho_old), state["rho_old"]) <= tol
    if not osp:  # rho^{n+1} is the static charge, bit for bit
        assert torch.equal(f.rho_old, f.rho_static)
    else:
        _compare_particles(el, osp[0], shape, wl.spacing, p.lengths, dtype, 1e-11 if dtype == "f64" else 2e-5,
                           1e-11 if dtype == "f64" else 2e-5)
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape_order", [1, 3])
def test_constant_weight_species(dtype, shape_order):
    """A species without a weight array (w = NULL) takes w_const for every particle: one call of three
    steps with the electrons and an immobile ion species both given that way gives bitwise the same
    fields, sources and particles as the same species with an explicit array of that weight (the
    particles as a set: the order inside a tile's run after regrouping is not unique)."""
    shape = (16, 16, 24)
    banner(f"pic_step with w_const species dtype={dtype} shape_order={shape_order}")
    wl = inputs.small(shape, ppc=2, shape_order=shape_order, center_order=8, dtype=dtype, u_th=0.2,
                      field_amp=0.05, seed=143)
    assert np.all(wl.electrons.w == wl.electrons.w[0]) and np.all(wl.ions.w == wl.ions.w[0])
    npd = np.float32 if dtype == "f32" else np.float64
    runs = []
    for constant in (False, True):
        ctx = piclib.Context.for_workload(wl, flags=0)
        f = ctx.fields_from_workload(wl)
        el = piclib.Species.from_host(wl.electrons, shape, dtype)
        ions = piclib.Species.from_host(wl.ions, shape, dtype)
        if constant:
            for sp, host in ((el, wl.electrons), (ions, wl.ions)):
                sp.w, sp.w_const = None, float(npd(host.w[0]))
        piclib.pic_deposit(ctx.ctx, [ions, el], f, piclib.PIC_DEP_RHO_ONLY)
        f.rho_old.copy_(f.rho_new)
        piclib.pic_step(ctx.ctx, f, [ions, el], 3)
        piclib.pic_sync(ctx.ctx)
        runs.append((ctx, f, el, ions))
    (_, fa, ea, ia), (_, fb, eb, ib) = runs
    for d in range(3):
        assert torch.equal(fa.E_stag[d], fb.E_stag[d]) and torch.equal(fa.B_stag[d], fb.B_stag[d]), d
        assert torch.equal(fa.J_nod[d], fb.J_nod[d]), d
    assert torch.equal(fa.rho_old, fb.rho_old)
    def records(sp):
        r = np.stack([np64(sp.cell)] + [np64(x) for x in sp.off] + [np64(x) for x in sp.u], axis=1)
        return r[np.lexsort(r.T[::-1])]

    for a, b in ((ea, eb), (ia, ib)):
        assert np.array_equal(records(a), records(b))
    for ctx, *_ in runs:
        ctx.close()
