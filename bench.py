#!/usr/bin/env python
"""Throughput of the hybrid nodal-staggered PSATD PIC step on one MI355X.

Workload (default, the largest configuration that fits one GPU): beam-driven wake on a
384x384x768 periodic grid (113,246,208 cells): cold plasma at 1 particle per cell (n0 = 2/256)
plus an electron drive beam (Gaussian, sigma_r = 8, sigma_z = 16 cells, gamma = 1000, 8 particles
per cell inside 3 sigma) with its relativistic self-fields, 114,172,416 macro-particles, immobile
ions as a static background, cubic B-spline shape, centering order 16, PSATD order 16,
c*dt = 0.5 cell, float32 fields and particles (FP64-built tables).  Synthetic and seeded
(paper_2106_12919_amd.inputs).

One "step" is one full hybrid cycle: staggered-to-nodal centering of E, B -> gather + Boris push
-> deposition of rho, J -> nodal-to-staggered centering of J -> forward FFTs of J, rho -> per-mode
PSATD update -> inverse FFTs of E, B.  The timed region is a single pic_step call of K steps with
every input resident in HBM (E, B stay in Fourier space between steps; the call's entry
transforms are inside the timed region).

Prints one JSON line.  Rates: particle-pushes/s = Np*K/T (``value``) and grid cell updates/s =
N*K/T.  ``roofline`` is the dominant stage's algorithmic bytes per launch over its mean duration,
timed with HIP events on the stream the library launches on.  ``lds_atomic_floor`` sets the
deposition's mean duration against the time its LDS atomics alone take at the rates a probe
measured on MI355X.  Further keys: ``fp64`` (the same workload in FP64, with the FP32 run's
field and energy error against it), ``thermal256_sweep`` (the 256^3 CIC thermal plasma at
centering orders 2..32 in FP32 and FP64, with the FP32 error against FP64 per order),
``fwd_bwd`` (forward + backward of the 64x64x128 laser workload, 60 steps, kinetic-energy loss)
and ``fwd_bwd_beam`` (of the beam-driven wake, beam-energy-loss objective), and
``cpu_baseline``: the FP64 NumPy oracle on the host cores on a bounded sample (two steps of the
beam-driven wake at 1/4 scale per axis; the particle part split over worker processes).
"""

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_HZ = 256, 2.4e9
# LDS atomic throughput (lane operations per second per CU) measured live by the library's probe
# (pic_probe_lds_atomics: the deposition's address patterns) at the start of the GPU part
LDS_RATES = {}


def deposit_lds_floor_ms(Np, shape_order, dtype, rate32, rate64, cus=CUS):
    """Time of the deposition's LDS atomics alone for Np particles depositing rho and J, at rate32
    and rate64 lane operations per second per compute unit: FP32 adds (J_x, J_y) as one 64-bit word
    and J_z, rho as 32-bit words per support node; FP64 adds four 64-bit words per node."""
    nodes = (2 if shape_order == 1 else 4) ** 3
    u64, u32 = (nodes, 2 * nodes) if dtype == "f32" else (4 * nodes, 0)
    return Np * (u64 / rate64 + u32 / rate32) / cus * 1e3


def traffic_profile(config_name, dtype):
    """The committed HBM-counter summary of a workload's bench command (FETCH_SIZE, WRITE_SIZE)."""
    return os.path.join(ROOT, "profiles", f"{config_name}_{dtype}_hbm_traffic.md")


def kernel_source_hash():
    """sha256 over the HIP sources: a recorded traffic figure is valid only for the sources it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_12919_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(stage, config_name="beam384", dtype="f32"):
    """Measured HBM bytes per launch of ``stage`` from the committed counter summary, or None
    when there is none or the kernel sources changed since the counters were taken."""
    try:
        text = open(traffic_profile(config_name, dtype)).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch", {}).get(stage)


CONFIG_TEXT = {
    "laser128": "laser128: 128x128x256 periodic, laser a0=2 lambda=16 waist=20 fwhm=30 into 2 ppc cold plasma "
                "(z>=64), cubic shape, centering order 16, PSATD order 16, c*dt=0.5",
    "laser64": "laser64: 64x64x128 periodic, laser a0=1 lambda=16 waist=12 fwhm=30 into 4 ppc cold plasma, "
               "cubic shape, centering order 8, PSATD order 16, c*dt=0.5",
    "thermal32": "thermal32: 32^3 periodic thermal plasma 8 ppc u_th=0.01, CIC, centering order 8, PSATD order 16",
    "thermal256": "thermal256: 256^3 periodic thermal plasma 8 ppc u_th=0.05, CIC, PSATD order 16",
    "beam384": "beam384: 384x384x768 periodic beam-driven wake, 1 ppc cold plasma n0=2/256 plus an electron beam "
               "sigma_r=8 sigma_z=16 gamma=1000 8 ppc inside 3 sigma with its self-fields, cubic shape, "
               "centering order 16, PSATD order 16, c*dt=0.5",
    "beam96": "beam96: the beam384 setup scaled by 1/4 per axis (96x96x192)",
}


def stage_bytes(stage, N, M, Np, s):
    """Algorithmic (compulsory) HBM bytes of one launch of a pic_step stage.

    N cells, M = nx*ny*(nz/2+1) half-spectrum modes, Np particles, s = sizeof(real)."""
    part_rw = 2 * (4 + 6 * s)          # cell + 3 offsets + 3 momenta, read and written
    part_r = 4 + 7 * s                 # cell, offsets, momenta, weight, read
    return {
        "center_s2n": 12 * N * s,      # 6 staggered components in, 6 nodal out
        "gather_push": 6 * N * s + Np * part_rw,
        "deposit": Np * part_r,        # particles read; the per-tile boxes are not algorithmic
        "deposit_reduce": 5 * N * s,   # rho, J written once; the static ion background read once
        "center_n2s": 6 * N * s,       # 3 in, 3 out
        "fft_forward": 4 * (N * s + M * 2 * s),          # J (3) and rho: real in, half spectrum out
        "psatd_update": M * (11 * 2 * s + 5 * s + 6 * 2 * s),  # 11 spectra + 5 tables in, 6 out
        "fft_inverse": 6 * (M * 2 * s + N * s),          # E, B: half spectrum in, real out
        "entry_forward": 7 * (N * s + M * 2 * s),
        "exit_inverse": 6 * (M * 2 * s + N * s),
        "tile_sort": Np * 12,          # full sort: cell read twice (count, rank), slot written
        "clear_sources": 0,            # only what no species wrote (the first species' reduction overwrites)
    }[stage]


# ------------------------------------------------------------------ CPU baseline (the oracle)

_CPU = {}  # what the worker processes of the CPU baseline inherit (set before the pool forks)


def _cpu_particle_part(k):
    """Worker k of the CPU baseline: gather + push and deposition of its slice of the particles."""
    from oracle import step as ostep
    c = _CPU
    n = c["sp"]["pos"].shape[0]
    sel = slice(k * n // c["workers"], (k + 1) * n // c["workers"])
    sp = {key: (val[sel] if key in ("pos", "u", "w") else val) for key, val in c["sp"].items()}
    sp["pos"], sp["u"] = sp["pos"].copy(), sp["u"].copy()
    v, pos_half = ostep.gather_push(sp, c["E_nod"], c["B_nod"], c["p"])
    rho = ostep.deposit_rho([sp], c["p"])
    J = ostep.deposit_current(sp, v, pos_half, c["p"])
    return rho, J, sp["pos"], sp["u"]


def cpu_workers():
    """The host cores of this GPU's share (at most 16, whatever the machine's total)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(config_name="beam96", steps=2, workers=None):
    """FP64 oracle on the host, timed over ``steps`` whole hybrid cycles of a bounded workload: the
    grid part (centering, transforms, field solve) in this process, the particle part (gather +
    push, deposition) split over ``workers`` forked processes.  Runs before anything touches the
    GPU (the workers are forked from this process)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    from oracle import step as ostep
    from paper_2106_12919_amd import inputs

    workers = workers or cpu_workers()
    wl = inputs.config(config_name, dtype="f64")
    p = ostep.Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    sp = {"pos": wl.electrons.positions(wl.spacing), "u": wl.electrons.u.copy(), "w": wl.electrons.w,
          "q": wl.electrons.q, "m": wl.electrons.m}
    ions = {"pos": wl.ions.positions(wl.spacing), "u": wl.ions.u, "w": wl.ions.w, "q": 1.0, "m": np.inf}
    rho_static = ostep.deposit_rho([ions], p)
    state = {"E_stag": [np.array(a) for a in wl.E], "B_stag": [np.array(a) for a in wl.B],
             "rho_old": ostep.deposit_rho([sp], p, rho_static)}
    ctx = mp.get_context("fork")
    ru = lambda: sum(getattr(resource.getrusage(w), f) for w in (resource.RUSAGE_SELF, resource.RUSAGE_CHILDREN)
                     for f in ("ru_utime", "ru_stime"))
    c0, t0 = ru(), time.perf_counter()
    for _ in range(steps):
        E_nod, B_nod = ostep.center_fields_s2n(state["E_stag"], state["B_stag"], p)
        _CPU.update(sp=sp, E_nod=E_nod, B_nod=B_nod, p=p, workers=workers)
        with ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            parts = list(ex.map(_cpu_particle_part, range(workers)))
        rho_new = rho_static + sum(q[0] for q in parts)
        J_nod = [sum(q[1][d] for q in parts) for d in range(3)]
        sp["pos"] = np.concatenate([q[2] for q in parts])
        sp["u"] = np.concatenate([q[3] for q in parts])
        J_stag = ostep.center_current_n2s(J_nod, p)
        E, B = ostep.push_fields(state["E_stag"], state["B_stag"], J_stag, state["rho_old"], rho_new, p)
        state = {"E_stag": E, "B_stag": B, "rho_old": rho_new}
    T, C = time.perf_counter() - t0, ru() - c0
    _CPU.clear()
    Np = wl.electrons.n
    return {
        "value": Np * steps / T, "unit": "particle-pushes/s", "cores": max(1, round(C / T)), "kind": "oracle",
        "sample": f"{steps} FP64 NumPy oracle steps of {config_name} ({wl.cells} cells, {Np} particles"
                  + ("; the beam-driven wake at 1/4 scale per axis, the same per-cell physics" if config_name ==
                     "beam96" else "") + f"), {T:.1f} s wall, {C:.1f} s CPU: grid part in one process, particle "
                  f"part over {workers} worker processes",
        "cell_updates_per_s": wl.cells * steps / T,
        "workers": workers,
    }


def cpu_single_thread(config_name, steps):
    """FP64 oracle in this process alone (one thread: NumPy's elementwise work and transforms run
    single-threaded), ``steps`` whole hybrid cycles of ``config_name``."""
    import numpy as np

    from oracle import step as ostep
    from paper_2106_12919_amd import inputs

    wl = inputs.config(config_name, dtype="f64")
    p = ostep.Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    sp = {"pos": wl.electrons.positions(wl.spacing), "u": wl.electrons.u.copy(), "w": wl.electrons.w,
          "q": wl.electrons.q, "m": wl.electrons.m}
    ions = {"pos": wl.ions.positions(wl.spacing), "u": wl.ions.u, "w": wl.ions.w, "q": 1.0, "m": np.inf}
    rho_static = ostep.deposit_rho([ions], p)
    state = {"E_stag": [np.array(a) for a in wl.E], "B_stag": [np.array(a) for a in wl.B],
             "rho_old": ostep.deposit_rho([sp], p, rho_static)}
    ru = lambda: sum(getattr(resource.getrusage(resource.RUSAGE_SELF), f) for f in ("ru_utime", "ru_stime"))
    c0, t0 = ru(), time.perf_counter()
    for _ in range(steps):
        ostep.step(state, [sp], p, rho_static)
    T, C = time.perf_counter() - t0, ru() - c0
    Np = wl.electrons.n
    return {"workload": config_name, "steps": steps, "value": Np * steps / T, "unit": "particle-pushes/s",
            "cell_updates_per_s": wl.cells * steps / T, "wall_s": round(T, 2), "cpu_s": round(C, 2),
            "cores": max(1, round(C / T))}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="beam384", choices=sorted(CONFIG_TEXT))
    ap.add_argument("--dtype", default=None, choices=["f32", "f64"])
    ap.add_argument("--center-order", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-config", default="beam96", choices=sorted(CONFIG_TEXT),
                    help="workload of the CPU oracle sample (default: the beam-driven wake at 1/4 scale)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of the main workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 256^3 thermal plasma at centering orders 2..32 in FP32 and FP64")
    ap.add_argument("--sweep-orders", default="2,4,8,16,32", metavar="LIST")
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--spectral-centering", action="store_true",
                    help="apply the finite-order centering as its Fourier symbol inside the per-mode update "
                         "(PIC_SPECTRAL_CENTERING; same results up to rounding, no real-space centering passes)")
    ap.add_argument("--nodal-solver", action="store_true",
                    help="the nodal comparison cycle (PIC_NODAL_SOLVER): fields on the nodes, centered [k]_c, "
                         "no centering")
    ap.add_argument("--staggered-cycle", action="store_true",
                    help="run the fully staggered comparison cycle (PIC_STAGGERED_CYCLE) instead of the hybrid one")
    ap.add_argument("--current-correction", action="store_true",
                    help="project J onto the continuity equation before each field solve (PIC_CURRENT_CORRECTION)")
    ap.add_argument("--field-adjoint", action="store_true",
                    help="also time psatd_push_fields and its reverse mode psatd_push_fields_adjoint "
                         "(\"field_solve\" in the JSON line)")
    ap.add_argument("--galilean", type=float, default=None, metavar="VZ",
                    help="also time the workload with the standard Galilean solver, v_gal = (0, 0, VZ) c")
    ap.add_argument("--averaged", action="store_true",
                    help="with --galilean: the averaged Galilean scheme (PIC_AVERAGED)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward+backward measurements (laser64 and the beam-driven wake)")
    ap.add_argument("--adjoint-config", default="laser64", choices=sorted(CONFIG_TEXT))
    ap.add_argument("--checkpoint-every", default="auto", metavar="K|auto",
                    help="checkpoint interval of the forward+backward legs; auto: every step when the "
                         "states fit in half the free device memory, else the smallest interval that fits")
    ap.add_argument("--adjoint-steps", type=int, default=0, metavar="K",
                    help="steps of the forward+backward run (default: the configuration's length)")
    ap.add_argument("--adjoint-reps", type=int, default=3)
    ap.add_argument("--beam-adjoint-steps", type=int, default=20,
                    help="steps of the beam-driven wake's forward+backward run (0: skip it)")
    ap.add_argument("--precision-statement", default="", metavar="LIST",
                    help="instead of timing: the FP32 error against the FP64 path over each listed workload's "
                         "full length (e.g. laser128,laser64,beam384,thermal256), fields, energy, momenta, charge")
    ap.add_argument("--precision-every", type=int, default=10, metavar="K",
                    help="with --precision-statement: steps per pic_step call, the errors taken after each call")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy a MIB-MiB float32 tensor 3 times (a plain copy kernel "
                         "of known size, the reference for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the hybrid PSATD step runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.precision_statement:
        import torch
        torch.cuda.set_device(0)
        out = {"precision_statement": [precision_statement(name, args.precision_every)
                                       for name in args.precision_statement.split(",")]}
        print(json.dumps(out))
        return

    cpu = None
    if not args.no_cpu_baseline:  # first: its worker processes fork from this one, before any GPU use
        print(f"[bench] timing the CPU oracle on {args.cpu_config} ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cpu_config)
        print(f"[bench] CPU oracle: {cpu['value']:.3e} pushes/s on {cpu['cores']} cores", file=sys.stderr,
              flush=True)
        # and on one thread, the two smallest configurations (thermal32 2 steps, laser64 1 step)
        cpu["single_thread"] = [cpu_single_thread("thermal32", 2), cpu_single_thread("laser64", 1)]

    import torch

    from paper_2106_12919_amd import inputs
    from paper_2106_12919_amd import lib as piclib

    torch.cuda.set_device(0)
    LDS_RATES[32] = piclib.pic_probe_lds_atomics(32, 4096)
    LDS_RATES[64] = piclib.pic_probe_lds_atomics(64, 4096)
    print(f"[bench] LDS atomics: {LDS_RATES[32] / CLOCK_HZ:.1f} (32-bit) and {LDS_RATES[64] / CLOCK_HZ:.1f} (64-bit) "
          f"lane-ops per clock per CU at {CLOCK_HZ / 1e9} GHz", file=sys.stderr, flush=True)
    wl = inputs.config(args.config, dtype=args.dtype, center_order=args.center_order)
    print(f"[bench] workload {args.config} dtype={wl.dtype} cells={wl.cells} particles={wl.electrons.n}",
          file=sys.stderr, flush=True)
    flags = ((piclib.PIC_SPECTRAL_CENTERING if args.spectral_centering else 0)
             | (piclib.PIC_NODAL_SOLVER if args.nodal_solver else 0)
             | (piclib.PIC_STAGGERED_CYCLE if args.staggered_cycle else 0)
             | (piclib.PIC_CURRENT_CORRECTION if args.current_correction else 0))
    keep = not args.no_fp64 and wl.dtype == "f32"
    result, final32 = run_gpu(wl, args.config, args.steps, args.warmup, args.calibrate_copy, flags, keep=keep)
    if keep:  # the same workload, steps and flags in FP64; the FP32 run's error against it
        wl.dtype = "f64"
        r64, final64 = run_gpu(wl, args.config, args.steps, args.warmup, 0, flags, keep=True)
        wl.dtype = "f32"
        result["fp64"] = {"value": r64["value"], "unit": "particle-pushes/s", "ms_per_step": r64["ms_per_step"],
                          "cell_updates_per_s": r64["cell_updates_per_s"], "roofline": r64["roofline"],
                          "stages": {k: v["ms_avg"] for k, v in r64["stages"].items()},
                          "fp32_error_vs_fp64": field_errors(final32, final64, wl.spacing,
                                                             steps=args.warmup + args.steps)}
        del final32, final64
        torch.cuda.empty_cache()
    # the roofline against the copy rate this GPU reaches as well as against the peak
    cb = copy_bandwidth()
    result["hbm_copy"] = cb
    result["roofline"]["frac_of_copy"] = round(result["roofline"]["achieved"] / cb["GBps"], 4)
    if args.field_adjoint:
        result["field_solve"] = time_field_solve(wl, flags)
    if args.galilean is not None:
        gflags = flags | (piclib.PIC_AVERAGED if args.averaged else 0)
        r, _ = run_gpu(wl, args.config, args.steps, args.warmup, 0, gflags, v_gal=(0.0, 0.0, args.galilean))
        M = wl.shape[0] * wl.shape[1] * (wl.shape[2] // 2 + 1)
        s = 4 if wl.dtype == "f32" else 8
        # 11 spectra and 6 complex tables in, 6 spectra out (averaged: 6 more tables, 6 more spectra out)
        upd = M * (11 * 2 * s + 12 * s + 6 * 2 * s) + (M * (12 * s + 6 * 2 * s) if args.averaged else 0)
        ms = r["stages"]["psatd_update"]["ms_avg"]
        result["galilean"] = {"v_gal": [0.0, 0.0, args.galilean], "averaged": bool(args.averaged),
                              "ms_per_step": r["ms_per_step"],
                              "value": r["value"], "stages": {k: v["ms_avg"] for k, v in r["stages"].items()},
                              "psatd_update_algo_bytes": upd, "psatd_update_GBps": round(upd / (ms * 1e-3) / 1e9, 1)}
    del wl
    if not args.no_sweep:
        orders = [int(x) for x in args.sweep_orders.split(",") if x]
        print(f"[bench] thermal256 at centering orders {orders}, FP32 and FP64 ...", file=sys.stderr, flush=True)
        result["thermal256_sweep"] = sweep_thermal256(orders, args.sweep_steps)
    if not args.no_adjoint:
        print(f"[bench] forward+backward of {args.adjoint_config} ...", file=sys.stderr, flush=True)
        result["fwd_bwd"] = time_fwd_bwd(args.adjoint_config, args.checkpoint_every, reps=args.adjoint_reps,
                                         steps=args.adjoint_steps)
        if args.beam_adjoint_steps > 0:
            print("[bench] forward+backward of beam384 (beam-energy-loss objective) ...", file=sys.stderr,
                  flush=True)
            result["fwd_bwd_beam"] = time_fwd_bwd("beam384", args.checkpoint_every, reps=1,
                                                  steps=args.beam_adjoint_steps, loss="beam_energy_loss")
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


def field_errors(a, b, spacing, steps):
    """FP32 fields ``a`` against FP64 fields ``b`` of the same run (dicts of E, B device tensors):
    the largest max-norm and L2 (Sec. 5.2 eq. L2_norm_error) relative error over the six
    components, and |W32 - W64| / W64 of the field energy (Sec. 2 item iii), accumulated in FP64."""
    import torch
    dV = spacing[0] * spacing[1] * spacing[2]
    worst_max = worst_l2 = 0.0
    W = [0.0, 0.0]
    for name in ("E", "B"):
        for x, y in zip(a[name], b[name]):
            x64 = x.double()
            d = x64 - y
            ymax = float(torch.max(torch.abs(y)))
            if ymax > 0:
                worst_max = max(worst_max, float(torch.max(torch.abs(d))) / ymax)
                worst_l2 = max(worst_l2, float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(y)))
            W[0] += float(torch.sum(x64 * x64))
            W[1] += float(torch.sum(y * y))
            del x64, d
    W = [0.5 * w * dV for w in W]
    return {"after_steps": steps, "field_max_rel": worst_max, "field_l2_rel": worst_l2,
            "W_rel": abs(W[0] - W[1]) / W[1] if W[1] > 0 else abs(W[0]), "reference": "the FP64 HIP path"}


def precision_statement(config_name, every=10):
    """FP32 against FP64 over a workload's full length, in pic_step calls of ``every`` steps (a call
    keeps E, B in Fourier space between its steps, as production runs do; each call adds one FP32
    round trip of the state): both runs keep the caller's particle order (PIC_KEEP_ORDER), so
    particles compare index by index.  After each call the worst max-norm and L2 relative field
    error over the six components, |W32 - W64| / W64, the momentum error max |u32 - u64| / max |u64|,
    and the electron charge error of the FP32 deposition |sum rho_e dV - sum q w| / |sum q w|; the
    worst of each over the run and the final values."""
    import torch

    from paper_2106_12919_amd import inputs
    from paper_2106_12919_amd import lib as piclib

    wl = inputs.config(config_name)
    orders = [2, 32] if config_name == "thermal256" else [wl.center_order]
    results = []
    for order in orders:
        wl.center_order = order
        runs = {}
        for dtype in ("f32", "f64"):
            wl.dtype = dtype
            ctx = piclib.Context.for_workload(wl, flags=piclib.PIC_KEEP_ORDER)
            f = ctx.fields_from_workload(wl)
            el = piclib.Species.from_host(wl.electrons, wl.shape, dtype)
            ions = piclib.Species.from_host(wl.ions, wl.shape, dtype)
            ctx.init_charge(f, el, ions)
            runs[dtype] = (ctx, f, el)
        q_el = -float(torch.sum(runs["f64"][2].w))
        dV = wl.spacing[0] * wl.spacing[1] * wl.spacing[2]
        rows = []
        for n0 in range(0, wl.steps, every):
            k = min(every, wl.steps - n0)
            n = n0 + k - 1
            for dtype in ("f32", "f64"):
                ctx, f, el = runs[dtype]
                piclib.pic_step(ctx.ctx, f, [el], k)
            torch.cuda.synchronize()
            (c32, f32, e32), (c64, f64, e64) = runs["f32"], runs["f64"]
            row = field_errors({"E": f32.E_stag, "B": f32.B_stag}, {"E": f64.E_stag, "B": f64.B_stag}, wl.spacing,
                               n + 1)
            umax = max(float(torch.max(torch.abs(t))) for t in e64.u)
            row["u_max_rel"] = max(float(torch.max(torch.abs(a.double() - b))) for a, b in zip(e32.u, e64.u)) / umax
            rho_e = f32.rho_old.double() - f32.rho_static.double()
            row["charge_rel"] = abs(float(torch.sum(rho_e)) * dV - q_el) / abs(q_el)
            rows.append(row)
            if (n + 1) % 50 == 0 or n + 1 == wl.steps:
                print(f"[precision] {config_name} order {order} step {n + 1}: |W32-W64|/W64 {row['W_rel']:.2e}, "
                      f"field max rel {row['field_max_rel']:.2e}", file=sys.stderr, flush=True)
        for dtype in ("f32", "f64"):
            runs[dtype][0].close()
        del runs
        torch.cuda.empty_cache()
        keys = ("field_max_rel", "field_l2_rel", "W_rel", "u_max_rel", "charge_rel")
        results.append({"workload": CONFIG_TEXT[config_name], "center_order": order, "steps": wl.steps,
                        "steps_per_call": every,
                        "worst": {k: max(r[k] for r in rows) for k in keys},
                        "final": {k: rows[-1][k] for k in keys}, "reference": "the FP64 HIP path"})
    return results


def sweep_thermal256(orders, steps, warmup=2):
    """The 256^3 thermal plasma (134,217,728 particles, CIC) at each centering order in FP32 and
    FP64: rates per dtype and order, and the FP32 run's field and energy error against the FP64 run
    of the same order after the same steps.  Particles are uploaded once per dtype and restored from
    a device copy before each run."""
    import torch

    from paper_2106_12919_amd import inputs
    from paper_2106_12919_amd import lib as piclib

    wl = inputs.config("thermal256")
    out = {"workload": CONFIG_TEXT["thermal256"], "steps": steps, "warmup": warmup, "orders": {}}
    dev = {}
    for dtype in ("f32", "f64"):
        el = piclib.Species.from_host(wl.electrons, wl.shape, dtype)
        ions = piclib.Species.from_host(wl.ions, wl.shape, dtype)
        dev[dtype] = (el, ions, el.cell.clone(), [t.clone() for t in el.off], [t.clone() for t in el.u],
                      el.w.clone())
    for order in orders:
        wl.center_order = order
        finals, row = {}, {}
        for dtype in ("f32", "f64"):
            el, ions, cell0, off0, u0, w0 = dev[dtype]
            el.cell.copy_(cell0)
            el.w.copy_(w0)
            for d in range(3):
                el.off[d].copy_(off0[d])
                el.u[d].copy_(u0[d])
            wl.dtype = dtype
            r, fin = run_gpu(wl, "thermal256", steps, warmup, 0, 0, keep=True, species=(el, ions))
            finals[dtype] = fin
            row[dtype] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                          "cell_updates_per_s": r["cell_updates_per_s"],
                          "stages": {k: v["ms_avg"] for k, v in r["stages"].items()},
                          "roofline": r["roofline"]}
            print(f"[sweep] order {order} {dtype}: {r['ms_per_step']:.3f} ms/step, {r['value']:.3e} pushes/s",
                  file=sys.stderr, flush=True)
        row["fp32_error_vs_fp64"] = field_errors(finals["f32"], finals["f64"], wl.spacing, steps + warmup)
        out["orders"][str(order)] = row
        del finals
        torch.cuda.empty_cache()
    return out


def time_field_solve(wl, flags, reps=20):
    """Mean ms of one psatd_push_fields and of one psatd_push_fields_adjoint on the workload grid
    (11 forward + 6 inverse transforms and the update; 6 forward + 11 inverse and the adjoint)."""
    import torch

    from paper_2106_12919_amd import lib as piclib

    ctx = piclib.Context.for_workload(wl, flags=flags)
    f = ctx.fields_from_workload(wl)
    out = {}
    for name, fn in (("forward_ms", piclib.psatd_push_fields), ("adjoint_ms", piclib.psatd_push_fields_adjoint)):
        fn(ctx.ctx, f)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn(ctx.ctx, f)
        t1.record()
        torch.cuda.synchronize()
        out[name] = round(t0.elapsed_time(t1) / reps, 4)
    ctx.close()
    out["adjoint_over_forward"] = round(out["adjoint_ms"] / out["forward_ms"], 3)
    return out


def time_fwd_bwd(config_name, every, reps=3, steps=0, loss="kinetic"):
    """Forward + backward of a differentiable run: ``steps`` of the config (default its length)
    through autograd.PicSteps with checkpoints every ``every`` steps ("auto": every step when the
    states fit in half the free device memory, else the smallest interval that fits; reported as
    ``checkpoint_every``), gradients w.r.t. the initial
    E, B and momenta; set against the same run of the production forward (pic_step, default flags).
    Losses: "kinetic", the total electron kinetic energy sum w (gamma - 1) at the end; and
    "beam_energy_loss", the drive beam's energy loss sum_beam w (gamma^0 - gamma^end) (the beam's
    particles follow the plasma's in the beam-driven wake's species).  Means of ``reps`` timed runs
    after one untimed run."""
    import torch

    from paper_2106_12919_amd import autograd as pag
    from paper_2106_12919_amd import inputs
    from paper_2106_12919_amd import lib as piclib

    wl = inputs.config(config_name)
    K = steps if steps > 0 else wl.steps
    n_beam_start = wl.ions.n if loss == "beam_energy_loss" else 0  # the ions neutralise the plasma only

    def setup(flags):
        ctx = piclib.Context.for_workload(wl, flags=flags)
        f = ctx.fields_from_workload(wl)
        el = piclib.Species.from_host(wl.electrons, wl.shape, wl.dtype)
        ions = piclib.Species.from_host(wl.ions, wl.shape, wl.dtype)
        ctx.init_charge(f, el, ions)
        return ctx, f, el

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    ctx0, f0, el0 = setup(0)
    state0 = ([t.clone() for t in f0.E_stag], [t.clone() for t in f0.B_stag], f0.rho_old.clone(),
              el0.cell.clone(), [t.clone() for t in el0.off], [t.clone() for t in el0.u], el0.w.clone())

    def forward_only():
        for d in range(3):
            f0.E_stag[d].copy_(state0[0][d])
            f0.B_stag[d].copy_(state0[1][d])
            el0.off[d].copy_(state0[4][d])
            el0.u[d].copy_(state0[5][d])
        f0.rho_old.copy_(state0[2])
        el0.cell.copy_(state0[3])
        el0.w.copy_(state0[6])
        piclib.pic_step(ctx0.ctx, f0, [el0], K)

    T_fwd = timed(forward_only)
    ctx0.close()
    del state0, f0, el0
    torch.cuda.empty_cache()
    ctx, f, el = setup(piclib.PIC_KEEP_ORDER)
    if every == "auto":  # store every state that fits in half the free memory
        free, _ = torch.cuda.mem_get_info()
        every = pag.checkpoint_interval(ctx, el.n, K, 0.5 * free)
    every = int(every)
    E_in, B_in, u_in = torch.stack(f.E_stag), torch.stack(f.B_stag), torch.stack(el.u)
    off_in = torch.stack(el.off)
    grads = {}
    wb = el.w[n_beam_start:]
    gamma0 = torch.sqrt(1 + torch.sum(u_in[:, n_beam_start:] ** 2, dim=0))

    def fwd_bwd():
        run = pag.DifferentiableRun(ctx, el.q, el.m, nsteps=K, checkpoint_every=every, rho_static=f.rho_static)
        E = E_in.clone().requires_grad_(True)
        B = B_in.clone().requires_grad_(True)
        u = u_in.clone().requires_grad_(True)
        out = pag.PicSteps.apply(run, el.cell, el.w, E, B, f.rho_old, off_in, u)
        uf = out[5]
        if loss == "kinetic":
            L = torch.sum(el.w * (torch.sqrt(1 + torch.sum(uf * uf, dim=0)) - 1))
        else:
            ub = uf[:, n_beam_start:]
            L = torch.sum(wb * (gamma0 - torch.sqrt(1 + torch.sum(ub * ub, dim=0))))
        L.backward()
        grads["loss"] = float(L.detach())
        grads["norm"] = float(torch.sqrt(torch.sum(E.grad ** 2) + torch.sum(B.grad ** 2) + torch.sum(u.grad ** 2)))

    T_fb = timed(fwd_bwd)
    piclib.pic_stage_times(ctx.ctx)  # reset
    piclib.pic_profile(ctx.ctx, True)
    fwd_bwd()
    torch.cuda.synchronize()
    stages = piclib.pic_stage_times(ctx.ctx)
    piclib.pic_profile(ctx.ctx, False)
    ctx.close()
    Np = wl.electrons.n
    what = ("sum w (gamma - 1) of all electrons at the end" if loss == "kinetic" else
            "beam energy loss sum_beam w (gamma^0 - gamma^end)")
    return {"workload": CONFIG_TEXT[config_name], "dtype": wl.dtype, "steps": K, "checkpoint_every": every,
            "loss": what + "; gradients w.r.t. initial E, B (Yee) and u",
            "forward_ms_per_step": round(1e3 * T_fwd / K, 4), "fwd_bwd_ms_per_step": round(1e3 * T_fb / K, 4),
            "fwd_bwd_over_forward": round(T_fb / T_fwd, 3),
            "fwd_bwd_particle_pushes_per_s": Np * K / T_fb, "fwd_bwd_cell_updates_per_s": wl.cells * K / T_fb,
            "loss_value": grads["loss"], "grad_norm": grads["norm"],
            "stage_ms_total_one_run": {k: round(v[0], 3) for k, v in stages.items() if v[1]}}


def copy_bandwidth(mib=1024, reps=5):
    """Device-to-device copy rate in GB/s (bytes read plus written), best of ``reps`` copies of a
    ``mib`` MiB buffer timed with events on the current stream: the HBM rate a streaming kernel
    reaches in practice, beside the 8 TB/s peak."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": round(2 * n * 4 / (best * 1e-3) / 1e9, 1), "bytes_per_copy": 2 * n * 4,
            "ms": round(best, 4), "kernel": "torch copy_ of a float32 buffer, best of %d" % reps}


def run_gpu(wl, config_name, steps, warmup, calibrate_copy, flags=0, v_gal=(0.0, 0.0, 0.0), keep=False,
            species=None):
    """Times ``steps`` hybrid cycles of the workload (one pic_step call) after ``warmup`` steps.

    Returns (result dict, final fields): with ``keep`` the final E_stag, B_stag as device tensors
    ({"E": [...], "B": [...]}), else None.  ``species``: already uploaded (electrons, ions)."""
    import torch

    from paper_2106_12919_amd import lib as piclib

    ctx = piclib.Context.for_workload(wl, flags=flags, v_gal=v_gal)
    f = ctx.fields_from_workload(wl)
    if species is None:
        el = piclib.Species.from_host(wl.electrons, wl.shape, wl.dtype)
        ions = piclib.Species.from_host(wl.ions, wl.shape, wl.dtype)
    else:
        el, ions = species
    ctx.init_charge(f, el, ions)
    del ions
    piclib.pic_step(ctx.ctx, f, [el], warmup)
    piclib.pic_sync(ctx.ctx)
    print(f"[bench] warmup {warmup} steps done", file=sys.stderr, flush=True)
    if calibrate_copy > 0:
        n = calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: 3 x {calibrate_copy} MiB", file=sys.stderr, flush=True)
        del src, dst

    piclib.pic_stage_times(ctx.ctx)  # reset
    piclib.pic_profile(ctx.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    piclib.pic_step(ctx.ctx, f, [el], steps)
    piclib.pic_sync(ctx.ctx)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    stages = piclib.pic_stage_times(ctx.ctx)
    piclib.pic_profile(ctx.ctx, False)
    W, Q = piclib.pic_diagnostics(ctx.ctx, f)
    print(f"[bench] timed {steps} steps in {T:.4f} s; field energy {W:.6e}, total charge {Q:.3e}",
          file=sys.stderr, flush=True)

    K = steps
    N = wl.cells
    M = wl.shape[0] * wl.shape[1] * (wl.shape[2] // 2 + 1)
    Np = el.n
    s = 4 if wl.dtype == "f32" else 8
    breakdown = {}
    ntiles = 1  # the library's particle tiles: 8 cells along each axis, partial ones at the upper ends
    for n in wl.shape:
        ntiles *= -(-n // 8)
    for name, (ms, cnt) in stages.items():
        if cnt == 0:
            continue
        avg = ms / cnt
        b = stage_bytes(name, N, M, Np, s)
        if name == "tile_sort":
            # only a call's first step sorts the particles; the later ones scan the tile counts the
            # previous deposition took and form each tile's 27 neighbour bases (counts, starts and
            # cursors, 27 counts read and 27 bases written: 236 bytes per tile)
            b = (b + (cnt - 1) * 236 * ntiles) // cnt
        breakdown[name] = {"ms_avg": round(avg, 5), "launches": cnt, "algo_bytes": b,
                           "GBps": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    dom = max((k for k in breakdown if k not in ("entry_forward", "exit_inverse")),
              key=lambda k: breakdown[k]["ms_avg"] * breakdown[k]["launches"])
    d = breakdown[dom]
    achieved = d["algo_bytes"] / (d["ms_avg"] * 1e-3) / 1e9
    lds_floor = None
    if "deposit" in breakdown and LDS_RATES:
        fl = deposit_lds_floor_ms(Np, wl.shape_order, wl.dtype, LDS_RATES[32], LDS_RATES[64])
        dep = breakdown["deposit"]["ms_avg"]
        lds_floor = {"kernel": "deposit", "bound": "lds_atomics", "floor_ms": round(fl, 5), "ms_per_launch": dep,
                     "frac": round(fl / dep, 4),
                     "basis": f"{LDS_RATES[32] / CLOCK_HZ:.2f} (u32) and {LDS_RATES[64] / CLOCK_HZ:.2f} (u64) "
                              f"lane-ops/clk/CU measured now by pic_probe_lds_atomics, {CUS} CUs at "
                              f"{CLOCK_HZ / 1e9} GHz"}
    final = None
    if keep:
        final = {"E": [t.clone() for t in f.E_stag], "B": [t.clone() for t in f.B_stag]}
    ctx.close()
    del f
    result = {
        "metric": "particle-pushes/s and grid-cell updates/s per PIC step, FP32 vs FP64, fwd and fwd+bwd",
        "value": Np * K / T,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": warmup,
        "ms_per_step": 1e3 * T / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.dtype,
        "data": "synthetic (seeded plasma, beam and laser workloads)",
        "config": {"workload": CONFIG_TEXT[config_name], "cells": N, "particles": Np,
                   "center_order": wl.center_order, "shape_order": wl.shape_order, "pass": "forward",
                   "centering": ("none (nodal solver)" if flags & piclib.PIC_NODAL_SOLVER else
                                 "none (staggered cycle)" if flags & piclib.PIC_STAGGERED_CYCLE else
                                 "spectral" if flags & piclib.PIC_SPECTRAL_CENTERING else "real-space"),
                   "current_correction": bool(flags & piclib.PIC_CURRENT_CORRECTION)},
        "cell_updates_per_s": N * K / T,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(dom, config_name, wl.dtype) if flags == 0 else None,
                     "algo_bytes_per_launch": d["algo_bytes"], "ms_per_launch": d["ms_avg"]},
        "lds_atomic_floor": lds_floor,
        "stages": breakdown,
    }
    return result, final


if __name__ == "__main__":
    main()
