#!/usr/bin/env python
"""Throughput of the hybrid nodal-staggered PSATD PIC step on one MI355X.

Workload (default): 128x128x256 periodic grid, Gaussian laser (wavelength 16
cells, a0 = 2, waist 20, FWHM duration 30, x-polarised, +z) entering a cold
electron plasma at 2 particles/cell for z >= 64 (6,291,456 macro-particles),
immobile ions as a static background, cubic B-spline shape, centering order 16,
PSATD order 16, c*dt = 0.5 cell, float32 fields and particles (FP64-built
tables).  Synthetic and seeded (paper_2106_12919_amd.inputs).

One "step" is one full hybrid cycle: staggered-to-nodal centering of E, B ->
gather + Boris push -> deposition of rho, J -> nodal-to-staggered centering of
J -> forward FFTs of J, rho -> per-mode PSATD update -> inverse FFTs of E, B.
The timed region is a single pic_step call of K steps with every input
resident in HBM (E, B stay in Fourier space between steps; the call's entry
transforms are inside the timed region).

Prints one JSON line.  Rates: particle-pushes/s = Np*K/T (``value``) and grid
cell updates/s = N*K/T.  ``roofline`` is the dominant stage's algorithmic bytes
per launch over its mean duration, timed with HIP events on the stream the
library launches on.  ``lds_atomic_floor`` sets the deposition's mean duration
against the time its LDS atomics alone take at the rates a probe measured on
MI355X (the deposition is bound by those, not by HBM).  ``cpu_baseline`` times the FP64 NumPy oracle on the host
on a bounded sample (the full grid part of one step plus 1/8 of the particles;
the particle part is scaled by 8, it is linear in the particle count).
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
# LDS atomic throughput per compute unit, lane operations per clock, measured on MI355X with a
# probe (1024 blocks x 256 threads, immediate offsets): ds_add_u32 with the 32 lanes of each
# half wave on distinct words modulo 32, ds_add_u64 with 16 lanes on distinct words modulo 16.
LDS_U32_LANE_OPS = 14.5
LDS_U64_LANE_OPS = 9.9
CUS, CLOCK_HZ = 256, 2.4e9


def deposit_lds_floor_ms(Np, shape_order, dtype):
    """Time of the deposition's LDS atomics alone for Np particles depositing rho and J: FP32 adds
    (J_x, J_y) as one 64-bit word and J_z, rho as 32-bit words per support node; FP64 adds four
    64-bit words per node."""
    nodes = (2 if shape_order == 1 else 4) ** 3
    u64, u32 = (nodes, 2 * nodes) if dtype == "f32" else (4 * nodes, 0)
    clocks_per_cu = Np * (u64 / LDS_U64_LANE_OPS + u32 / LDS_U32_LANE_OPS) / CUS
    return clocks_per_cu / CLOCK_HZ * 1e3


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "laser128_f32_hbm_traffic.md")


def kernel_source_hash():
    """sha256 over the HIP sources: a recorded traffic figure is valid only for the sources it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_12919_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(stage):
    """Measured HBM bytes per launch of ``stage`` from the committed counter summary, or None
    when there is none or the kernel sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
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
        "tile_sort": Np * 12,          # cell read twice (count, rank), slot written
        "clear_sources": 0,            # only what no species wrote (the first species' reduction overwrites)
    }[stage]


def cpu_baseline(wl, Np):
    """FP64 oracle on the host: grid part of one step + 1/8 of the particles, particle part scaled by 8."""
    import numpy as np

    from oracle import step as ostep

    p = ostep.Params(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order)
    frac = 8
    sel = slice(0, wl.electrons.n // frac)
    sp = {"pos": wl.electrons.positions(wl.spacing)[sel], "u": wl.electrons.u[sel].copy(),
          "w": wl.electrons.w[sel], "q": wl.electrons.q, "m": wl.electrons.m}
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    E_nod, B_nod = ostep.center_fields_s2n(wl.E, wl.B, p)
    t1 = time.perf_counter()
    v, pos_half = ostep.gather_push(sp, E_nod, B_nod, p)
    rho_new = ostep.deposit_rho([sp], p)
    J_nod = ostep.deposit_current(sp, v, pos_half, p)
    t2 = time.perf_counter()
    J_stag = ostep.center_current_n2s(J_nod, p)
    ostep.push_fields(wl.E, wl.B, J_stag, np.zeros(wl.shape), rho_new, p)
    t3 = time.perf_counter()
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    grid_s = (t1 - t0) + (t3 - t2)
    part_s = (t2 - t1) * frac
    step_s = grid_s + part_s
    cpu_s = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    cores = max(1, round(cpu_s / (t3 - t0)))
    return {
        "value": Np / step_s, "unit": "particle-pushes/s", "cores": cores, "kind": "oracle",
        "sample": f"one FP64 NumPy oracle step: full grid part ({grid_s:.1f} s) + particle part on "
                  f"{wl.electrons.n // frac} of {wl.electrons.n} electrons ({t2 - t1:.1f} s, scaled x{frac}); "
                  f"{step_s:.1f} s per step",
        "cell_updates_per_s": wl.cells / step_s,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="laser128", choices=sorted(CONFIG_TEXT))
    ap.add_argument("--dtype", default=None, choices=["f32", "f64"])
    ap.add_argument("--center-order", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-center-orders", default="", metavar="LIST",
                    help="after the main measurement, time the same workload at each centering order of the "
                         "comma-separated LIST ([sweep] lines on stderr, and JSON lines into --extra-json)")
    ap.add_argument("--extra-json", default="", metavar="PATH")
    ap.add_argument("--spectral-centering", action="store_true",
                    help="apply the finite-order centering as its Fourier symbol inside the per-mode update "
                         "(PIC_SPECTRAL_CENTERING; same results up to rounding, no real-space centering passes)")
    ap.add_argument("--nodal-solver", action="store_true",
                    help="the nodal comparison cycle (PIC_NODAL_SOLVER): fields on the nodes, centered [k]_c, "
                         "no centering")
    ap.add_argument("--staggered-cycle", action="store_true",
                    help="run the fully staggered comparison cycle (PIC_STAGGERED_CYCLE) instead of the hybrid one")
    ap.add_argument("--field-adjoint", action="store_true",
                    help="also time psatd_push_fields and its reverse mode psatd_push_fields_adjoint "
                         "(\"field_solve\" in the JSON line)")
    ap.add_argument("--galilean", type=float, default=None, metavar="VZ",
                    help="also time the workload with the standard Galilean solver, v_gal = (0, 0, VZ) c")
    ap.add_argument("--averaged", action="store_true",
                    help="with --galilean: the averaged Galilean scheme (PIC_AVERAGED)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward+backward measurement of the differentiable workload (laser64, FP32, "
                         "60 steps, kinetic-energy loss, checkpoints every 10 steps)")
    ap.add_argument("--adjoint-config", default="laser64", choices=sorted(CONFIG_TEXT))
    ap.add_argument("--checkpoint-every", type=int, default=10)
    ap.add_argument("--adjoint-steps", type=int, default=0, metavar="K",
                    help="steps of the forward+backward run (default: the configuration's length)")
    ap.add_argument("--adjoint-reps", type=int, default=3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy a MIB-MiB float32 tensor 3 times (a plain copy kernel "
                         "of known size, the reference for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs the hybrid PSATD step on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is described in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_12919_amd import inputs

    torch.cuda.set_device(0)
    wl = inputs.config(args.config, dtype=args.dtype, center_order=args.center_order)
    print(f"[bench] workload {args.config} dtype={wl.dtype} cells={wl.cells} particles={wl.electrons.n}",
          file=sys.stderr, flush=True)
    # PIC_SPECTRAL_CENTERING, PIC_NODAL_SOLVER, PIC_STAGGERED_CYCLE
    flags = (1 if args.spectral_centering else 0) | (2 if args.nodal_solver else 0) | (16 if args.staggered_cycle else 0)
    result = run_gpu(wl, args.config, args.steps, args.warmup, args.calibrate_copy, flags)
    if args.field_adjoint:
        result["field_solve"] = time_field_solve(wl, flags)
    if args.galilean is not None:
        gflags = flags | (8 if args.averaged else 0)  # PIC_AVERAGED
        r = run_gpu(wl, args.config, args.steps, args.warmup, 0, gflags, v_gal=(0.0, 0.0, args.galilean))
        M = wl.shape[0] * wl.shape[1] * (wl.shape[2] // 2 + 1)
        s = 4 if wl.dtype == "f32" else 8
        # 11 spectra and 6 complex tables in, 6 spectra out (averaged: 6 more tables, 6 more spectra out)
        upd = M * (11 * 2 * s + 12 * s + 6 * 2 * s) + (M * (12 * s + 6 * 2 * s) if args.averaged else 0)
        ms = r["stages"]["psatd_update"]["ms_avg"]
        result["galilean"] = {"v_gal": [0.0, 0.0, args.galilean], "averaged": bool(args.averaged),
                              "ms_per_step": r["ms_per_step"],
                              "value": r["value"], "stages": {k: v["ms_avg"] for k, v in r["stages"].items()},
                              "psatd_update_algo_bytes": upd, "psatd_update_GBps": round(upd / (ms * 1e-3) / 1e9, 1)}
    if not args.no_adjoint:
        print(f"[bench] forward+backward of {args.adjoint_config} ...", file=sys.stderr, flush=True)
        result["fwd_bwd"] = time_fwd_bwd(args.adjoint_config, args.checkpoint_every, reps=args.adjoint_reps,
                                         steps=args.adjoint_steps)
    if args.sweep_center_orders:
        for order in [int(x) for x in args.sweep_center_orders.split(",")]:
            wl.center_order = order
            r = run_gpu(wl, args.config, args.steps, args.warmup, 0, flags)
            line = {"sweep": "center_order", "center_order": order, "dtype": wl.dtype, "value": r["value"],
                    "ms_per_step": r["ms_per_step"], "cell_updates_per_s": r["cell_updates_per_s"],
                    "stages": {k: v["ms_avg"] for k, v in r["stages"].items()}}
            print("[sweep] " + json.dumps(line), file=sys.stderr, flush=True)
            if args.extra_json:
                with open(args.extra_json, "a") as fh:
                    fh.write(json.dumps(line) + "\n")
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl, result["config"]["particles"])
    print(json.dumps(result))


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


def time_fwd_bwd(config_name, every, reps=3, steps=0):
    """Forward + backward of the differentiable workload: its full run (``steps`` of the config)
    through autograd.PicSteps with checkpoints every ``every`` steps, the loss being the total
    electron kinetic energy sum w (gamma - 1) at the end, gradients w.r.t. the initial E, B and
    momenta; set against the same run of the production forward (pic_step, default flags).
    Means of ``reps`` timed runs after one untimed run."""
    import torch

    from paper_2106_12919_amd import autograd as pag
    from paper_2106_12919_amd import inputs
    from paper_2106_12919_amd import lib as piclib

    wl = inputs.config(config_name)
    K = steps if steps > 0 else wl.steps

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
              el0.cell.clone(), [t.clone() for t in el0.off], [t.clone() for t in el0.u])

    def forward_only():
        for d in range(3):
            f0.E_stag[d].copy_(state0[0][d])
            f0.B_stag[d].copy_(state0[1][d])
            el0.off[d].copy_(state0[4][d])
            el0.u[d].copy_(state0[5][d])
        f0.rho_old.copy_(state0[2])
        el0.cell.copy_(state0[3])
        piclib.pic_step(ctx0.ctx, f0, [el0], K)

    T_fwd = timed(forward_only)
    ctx0.close()
    ctx, f, el = setup(piclib.PIC_KEEP_ORDER)
    E_in, B_in, u_in = torch.stack(f.E_stag), torch.stack(f.B_stag), torch.stack(el.u)
    off_in = torch.stack(el.off)
    grads = {}

    def fwd_bwd():
        run = pag.DifferentiableRun(ctx, el.q, el.m, nsteps=K, checkpoint_every=every, rho_static=f.rho_static)
        E = E_in.clone().requires_grad_(True)
        B = B_in.clone().requires_grad_(True)
        u = u_in.clone().requires_grad_(True)
        out = pag.PicSteps.apply(run, el.cell, el.w, E, B, f.rho_old, off_in, u)
        uf = out[5]
        loss = torch.sum(el.w * (torch.sqrt(1 + torch.sum(uf * uf, dim=0)) - 1))
        loss.backward()
        grads["loss"] = float(loss.detach())
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
    return {"workload": CONFIG_TEXT[config_name], "dtype": wl.dtype, "steps": K, "checkpoint_every": every,
            "loss": "sum w (gamma - 1) at the end; gradients w.r.t. initial E, B (Yee) and u",
            "forward_ms_per_step": round(1e3 * T_fwd / K, 4), "fwd_bwd_ms_per_step": round(1e3 * T_fb / K, 4),
            "fwd_bwd_over_forward": round(T_fb / T_fwd, 3),
            "fwd_bwd_particle_pushes_per_s": Np * K / T_fb, "fwd_bwd_cell_updates_per_s": wl.cells * K / T_fb,
            "loss_value": grads["loss"], "grad_norm": grads["norm"],
            "stage_ms_total_one_run": {k: round(v[0], 3) for k, v in stages.items() if v[1]}}


def run_gpu(wl, config_name, steps, warmup, calibrate_copy, flags=0, v_gal=(0.0, 0.0, 0.0)):
    """Times ``steps`` hybrid cycles of the workload (one pic_step call) after ``warmup`` steps."""
    import torch

    from paper_2106_12919_amd import lib as piclib

    ctx = piclib.Context.for_workload(wl, flags=flags, v_gal=v_gal)
    f = ctx.fields_from_workload(wl)
    el = piclib.Species.from_host(wl.electrons, wl.shape, wl.dtype)
    ions = piclib.Species.from_host(wl.ions, wl.shape, wl.dtype)
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
    for name, (ms, cnt) in stages.items():
        if cnt == 0:
            continue
        avg = ms / cnt
        b = stage_bytes(name, N, M, Np, s)
        breakdown[name] = {"ms_avg": round(avg, 5), "launches": cnt, "algo_bytes": b,
                           "GBps": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    dom = max((k for k in breakdown if k not in ("entry_forward", "exit_inverse")),
              key=lambda k: breakdown[k]["ms_avg"] * breakdown[k]["launches"])
    d = breakdown[dom]
    achieved = d["algo_bytes"] / (d["ms_avg"] * 1e-3) / 1e9
    lds_floor = None
    if "deposit" in breakdown:
        fl = deposit_lds_floor_ms(Np, wl.shape_order, wl.dtype)
        dep = breakdown["deposit"]["ms_avg"]
        lds_floor = {"kernel": "deposit", "bound": "lds_atomics", "floor_ms": round(fl, 5), "ms_per_launch": dep,
                     "frac": round(fl / dep, 4),
                     "basis": f"{LDS_U32_LANE_OPS} (u32) and {LDS_U64_LANE_OPS} (u64) lane-ops/clk/CU measured, "
                              f"{CUS} CUs at {CLOCK_HZ / 1e9} GHz"}
    ctx.close()
    return {
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
        "data": "synthetic (seeded laser + plasma workload)",
        "config": {"workload": CONFIG_TEXT[config_name], "cells": N, "particles": Np,
                   "center_order": wl.center_order, "shape_order": wl.shape_order, "pass": "forward",
                   "centering": ("none (nodal solver)" if flags & 2 else
                                 "none (staggered cycle)" if flags & 16 else
                                 "spectral" if flags & 1 else "real-space")},
        "cell_updates_per_s": N * K / T,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(dom) if (config_name == "laser128" and wl.dtype == "f32") else None,
                     "algo_bytes_per_launch": d["algo_bytes"], "ms_per_launch": d["ms_avg"]},
        "lds_atomic_floor": lds_floor,
        "stages": breakdown,
    }


if __name__ == "__main__":
    main()
