"""ctypes binding of libpic (include/pic.h): argument marshalling only.

Every step of the hybrid PSATD cycle runs in the HIP library; this module only
turns torch tensors into the C structures and raises ``RuntimeError`` with the
library's message when a call fails.  The library must have been built
(``paper_2106_12919_amd.build``); there is no fallback.
"""

import ctypes
import math
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_uint32, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PIC_LIBRARY may name another build of the same sources (A/B timing of build variants).
LIB_PATH = os.environ.get("PIC_LIBRARY") or os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_EUNSUPPORTED, PIC_EHIP, PIC_ENOMEM, PIC_ESTATE = range(6)
PIC_F32, PIC_F64 = 0, 1
PIC_N2S, PIC_S2N = 0, 1
PIC_J, PIC_E, PIC_B = 0, 1, 2
PIC_DEP_RHO_AND_J, PIC_DEP_RHO_ONLY = 0, 1
PIC_CURRENT_CORRECTION = 1 << 0
PIC_DETERMINISTIC = 1 << 1
PIC_SPECTRAL_CENTERING = 1 << 2
PIC_NODAL_SOLVER = 1 << 3
PIC_KEEP_ORDER = 1 << 4
PIC_AVERAGED = 1 << 5
PIC_STAGGERED_CYCLE = 1 << 6


class pic_params(Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("dx", c_double), ("dy", c_double), ("dz", c_double), ("dt", c_double),
                ("shape_order", c_int32), ("center_order", c_int32), ("psatd_order", c_int32),
                ("dtype", c_int), ("flags", c_uint32), ("v_gal", c_double * 3)]


class pic_species(Structure):
    _fields_ = [("n", c_int64), ("cell", c_void_p), ("off", c_void_p * 3), ("u", c_void_p * 3),
                ("w", c_void_p), ("w_const", c_double), ("q", c_double), ("m", c_double)]


class pic_fields(Structure):
    _fields_ = [("E_stag", c_void_p * 3), ("B_stag", c_void_p * 3), ("E_nod", c_void_p * 3),
                ("B_nod", c_void_p * 3), ("J_nod", c_void_p * 3), ("J_stag", c_void_p * 3),
                ("rho_old", c_void_p), ("rho_new", c_void_p), ("rho_static", c_void_p),
                ("E_avg", c_void_p * 3), ("B_avg", c_void_p * 3)]


class pic_species_adjoint(Structure):
    _fields_ = [("off", c_void_p * 3), ("u", c_void_p * 3)]


_lib = None


def load():
    """Load libpic.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpic.so not found at {LIB_PATH}: build it with `python -m paper_2106_12919_amd.build`")
    # torch first: libpic must bind to the HIP runtime torch already uses (same soname),
    # so that torch's streams and device pointers are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "pic_init": (c_int, [POINTER(pic_params), c_void_p, POINTER(c_void_p)]),
        "pic_destroy": (c_int, [c_void_p]),
        "pic_set_stream": (c_int, [c_void_p, c_void_p]),
        "pic_deposit": (c_int, [c_void_p, POINTER(pic_species), c_int, POINTER(pic_fields), c_int]),
        "pic_deposit_noalloc": (c_int, [c_void_p, POINTER(pic_species), c_int, POINTER(pic_fields), c_int]),
        "pic_center": (c_int, [c_void_p, c_int, c_int, POINTER(pic_fields)]),
        "psatd_push_fields": (c_int, [c_void_p, POINTER(pic_fields)]),
        "psatd_push_fields_adjoint": (c_int, [c_void_p, POINTER(pic_fields)]),
        "pic_gather_push": (c_int, [c_void_p, POINTER(pic_fields), POINTER(pic_species), c_int]),
        "pic_step": (c_int, [c_void_p, POINTER(pic_fields), POINTER(pic_species), c_int, c_int]),
        "pic_step_adjoint": (c_int, [c_void_p, POINTER(pic_fields), POINTER(pic_species), c_int,
                                     POINTER(pic_fields), POINTER(pic_species_adjoint)]),
        "pic_sync": (c_int, [c_void_p]),
        "pic_diagnostics": (c_int, [c_void_p, POINTER(pic_fields), POINTER(c_double)]),
        "pic_gauss_residual": (c_int, [c_void_p, POINTER(pic_fields), POINTER(c_double)]),
        "pic_continuity_residual": (c_int, [c_void_p, POINTER(pic_fields), POINTER(c_double)]),
        "pic_profile": (c_int, [c_void_p, c_int]),
        "pic_stage_times": (c_int, [c_void_p, POINTER(c_double), POINTER(c_int64), c_int]),
        "pic_stage_name": (c_char_p, [c_int]),
        "pic_num_stages": (c_int, []),
        "pic_last_error": (c_char_p, [c_void_p]),
        "pic_strerror": (c_char_p, [c_int]),
        "pic_modified_wavenumber": (c_int, [ctypes.c_int32, c_double, ctypes.c_int32, ctypes.c_int32,
                                            POINTER(c_double)]),
        "pic_centering_factor": (c_int, [ctypes.c_int32, ctypes.c_int32, POINTER(c_double)]),
        "pic_stencil_extent": (c_int, [POINTER(pic_params), ctypes.c_int32, ctypes.c_int32, POINTER(c_double)]),
        "pic_probe_lds_atomics": (c_int, [c_int, c_int, POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, ctx=None):
    if status != PIC_OK:
        lib = load()
        msg = lib.pic_last_error(ctx).decode()
        raise RuntimeError(f"libpic: {lib.pic_strerror(status).decode()} ({status}): {msg}")


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ C-ABI mirrors (same names)

def pic_init(params, stream=None):
    ctx = c_void_p()
    st = load().pic_init(ctypes.byref(params), stream if stream is not None else _stream(), ctypes.byref(ctx))
    _check(st, None)
    return ctx


def pic_destroy(ctx):
    _check(load().pic_destroy(ctx))


def pic_set_stream(ctx, stream=None):
    _check(load().pic_set_stream(ctx, stream if stream is not None else _stream()), ctx)


def _species_array(species):
    arr = (pic_species * max(1, len(species)))()
    for i, s in enumerate(species):
        arr[i] = s.struct()
    return arr


def pic_deposit(ctx, species, fields, mode=PIC_DEP_RHO_AND_J):
    arr = _species_array(species)
    _check(load().pic_deposit(ctx, arr, len(species), ctypes.byref(fields.struct()), mode), ctx)


def pic_deposit_noalloc(ctx, species, fields, mode=PIC_DEP_RHO_AND_J):
    arr = _species_array(species)
    _check(load().pic_deposit_noalloc(ctx, arr, len(species), ctypes.byref(fields.struct()), mode), ctx)


def pic_center(ctx, direction, what, fields):
    _check(load().pic_center(ctx, direction, what, ctypes.byref(fields.struct())), ctx)


def psatd_push_fields(ctx, fields):
    _check(load().psatd_push_fields(ctx, ctypes.byref(fields.struct())), ctx)


def psatd_push_fields_adjoint(ctx, fields):
    _check(load().psatd_push_fields_adjoint(ctx, ctypes.byref(fields.struct())), ctx)


def pic_gather_push(ctx, fields, species):
    arr = _species_array(species)
    _check(load().pic_gather_push(ctx, ctypes.byref(fields.struct()), arr, len(species)), ctx)


def pic_step(ctx, fields, species, nsteps=1):
    arr = _species_array(species)
    _check(load().pic_step(ctx, ctypes.byref(fields.struct()), arr, len(species), nsteps), ctx)


def pic_step_adjoint(ctx, fields, species, adj_fields, adj_species):
    """Reverse mode of one step: ``adj_species`` is a list of SpeciesAdjoint (same order as ``species``)."""
    arr = _species_array(species)
    aarr = (pic_species_adjoint * max(1, len(adj_species)))()
    for i, a in enumerate(adj_species):
        aarr[i] = a.struct()
    _check(load().pic_step_adjoint(ctx, ctypes.byref(fields.struct()), arr, len(species),
                                   ctypes.byref(adj_fields.struct()), aarr), ctx)


def pic_sync(ctx):
    _check(load().pic_sync(ctx), ctx)


def pic_diagnostics(ctx, fields):
    out = (c_double * 2)()
    _check(load().pic_diagnostics(ctx, ctypes.byref(fields.struct()), out), ctx)
    return float(out[0]), float(out[1])


def pic_gauss_residual(ctx, fields):
    out = c_double()
    _check(load().pic_gauss_residual(ctx, ctypes.byref(fields.struct()), ctypes.byref(out)), ctx)
    return float(out.value)


def pic_continuity_residual(ctx, fields):
    out = c_double()
    _check(load().pic_continuity_residual(ctx, ctypes.byref(fields.struct()), ctypes.byref(out)), ctx)
    return float(out.value)


def pic_profile(ctx, enable=True):
    _check(load().pic_profile(ctx, 1 if enable else 0), ctx)


def pic_stage_times(ctx):
    lib = load()
    n = lib.pic_num_stages()
    ms = (c_double * n)()
    cnt = (c_int64 * n)()
    _check(lib.pic_stage_times(ctx, ms, cnt, n), ctx)
    return {lib.pic_stage_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}


def pic_modified_wavenumber(n, d, order, kind):
    """[k]_s (kind 0) or [k]_c (kind 1) at the DFT indices of an n-point axis (host, FP64)."""
    out = (c_double * n)()
    _check(load().pic_modified_wavenumber(n, d, order, kind, out))
    return [float(x) for x in out]


def pic_centering_factor(n, center_order):
    """zeta(k) of the centering of order center_order at the DFT indices of an n-point axis (host, FP64)."""
    out = (c_double * n)()
    _check(load().pic_centering_factor(n, center_order, out))
    return [float(x) for x in out]


def pic_stencil_extent(params, axis, coefficient):
    """Gamma(x_j), j = 0..n_axis-1, of PSATD coefficient (0 C, 1 S/w, 2 X1, 3 X2, 4 X3) along axis."""
    n = (params.nx, params.ny, params.nz)[axis]
    out = (c_double * n)()
    _check(load().pic_stencil_extent(ctypes.byref(params), axis, coefficient, out))
    return [float(x) for x in out]


def pic_probe_lds_atomics(width_bits, iters=4096):
    """Lane operations per second per compute unit of 32- or 64-bit integer LDS atomics."""
    out = c_double()
    _check(load().pic_probe_lds_atomics(width_bits, iters, ctypes.byref(out)))
    return out.value


# ------------------------------------------------------------------ tensor containers

class Species:
    """One species as separate contiguous device tensors (cell int32, off/u/w of the run dtype); with
    ``w`` None every particle has the weight ``w_const``."""

    def __init__(self, cell, off, u, w, q, m, w_const=0.0):
        self.cell, self.off, self.u, self.w, self.q, self.m = cell, list(off), list(u), w, float(q), float(m)
        self.w_const = float(w_const)

    @classmethod
    def from_host(cls, sp, shape, dtype, device="cuda"):
        import torch
        td = torch.float32 if dtype == "f32" else torch.float64
        nx, ny, nz = shape
        lin = ((sp.cell[:, 0] * ny + sp.cell[:, 1]) * nz + sp.cell[:, 2]).astype(np.int32)
        cell = torch.from_numpy(lin).to(device)
        npd = np.float32 if dtype == "f32" else np.float64
        off = []
        for d in range(3):
            o = sp.off[:, d].astype(npd)
            # an offset that rounds up to 1 in the run precision stays just below it
            o = np.where(o >= 1, np.nextafter(npd(1), npd(0)), o).astype(npd)
            off.append(torch.from_numpy(np.ascontiguousarray(o)).to(device))
        u = [torch.from_numpy(np.ascontiguousarray(sp.u[:, d])).to(device=device, dtype=td) for d in range(3)]
        w = torch.from_numpy(np.ascontiguousarray(sp.w)).to(device=device, dtype=td)
        return cls(cell, off, u, w, sp.q, sp.m)

    @property
    def n(self):
        return int(self.cell.numel())

    def struct(self):
        s = pic_species()
        s.n = self.n
        s.cell = _ptr(self.cell)
        for d in range(3):
            s.off[d] = _ptr(self.off[d])
            s.u[d] = _ptr(self.u[d])
        s.w = _ptr(self.w)
        s.w_const = self.w_const
        s.q, s.m = self.q, self.m
        return s

    def positions(self, shape, spacing):
        """(Np, 3) float64 host positions (for comparisons)."""
        nx, ny, nz = shape
        c = self.cell.cpu().numpy().astype(np.int64)
        idx = np.stack([c // (ny * nz), (c // nz) % ny, c % nz], axis=1)
        off = np.stack([o.cpu().numpy().astype(np.float64) for o in self.off], axis=1)
        return (idx + off) * np.asarray(spacing)[None, :]


class SpeciesAdjoint:
    """dL/d offsets (cells) and dL/du of one species: 3 + 3 contiguous device tensors."""

    def __init__(self, off, u):
        self.off, self.u = list(off), list(u)

    def struct(self):
        s = pic_species_adjoint()
        for d in range(3):
            s.off[d] = _ptr(self.off[d])
            s.u[d] = _ptr(self.u[d])
        return s


class Fields:
    """All grid arrays of a step as device tensors of the run dtype."""

    NAMES3 = ("E_stag", "B_stag", "E_nod", "B_nod", "J_nod", "J_stag")

    def __init__(self, shape, dtype, device="cuda", averaged=False):
        import torch
        td = torch.float32 if dtype == "f32" else torch.float64
        self.shape, self.dtype = tuple(shape), dtype
        for name in self.NAMES3:
            setattr(self, name, [torch.zeros(shape, dtype=td, device=device) for _ in range(3)])
        self.rho_old = torch.zeros(shape, dtype=td, device=device)
        self.rho_new = torch.zeros(shape, dtype=td, device=device)
        self.rho_static = None
        # averaged fields (PIC_AVERAGED)
        self.E_avg = [torch.zeros(shape, dtype=td, device=device) for _ in range(3)] if averaged else None
        self.B_avg = [torch.zeros(shape, dtype=td, device=device) for _ in range(3)] if averaged else None

    def struct(self):
        f = pic_fields()
        for name in self.NAMES3:
            arr = getattr(f, name)
            for d, t in enumerate(getattr(self, name)):
                arr[d] = _ptr(t)
        f.rho_old = _ptr(self.rho_old)
        f.rho_new = _ptr(self.rho_new)
        f.rho_static = _ptr(self.rho_static)
        for d in range(3):
            f.E_avg[d] = _ptr(self.E_avg[d]) if self.E_avg else None
            f.B_avg[d] = _ptr(self.B_avg[d]) if self.B_avg else None
        return f


def make_params(shape, spacing, dt, shape_order, center_order, psatd_order, dtype, flags=0, v_gal=(0.0, 0.0, 0.0)):
    p = pic_params()
    p.nx, p.ny, p.nz = shape
    p.dx, p.dy, p.dz = spacing
    p.dt = dt
    p.shape_order, p.center_order, p.psatd_order = shape_order, center_order, psatd_order
    p.dtype = PIC_F32 if dtype == "f32" else PIC_F64
    p.flags = flags
    for d in range(3):
        p.v_gal[d] = float(v_gal[d])
    return p


class Context:
    """Owns a pic_ctx for one workload; thin convenience over the C ABI."""

    def __init__(self, shape, spacing, dt, shape_order, center_order, psatd_order, dtype, stream=None, flags=0,
                 v_gal=(0.0, 0.0, 0.0)):
        self.params = make_params(shape, spacing, dt, shape_order, center_order, psatd_order, dtype, flags, v_gal)
        self.shape, self.spacing, self.dt, self.dtype = tuple(shape), tuple(spacing), dt, dtype
        self.ctx = pic_init(self.params, stream)

    @classmethod
    def for_workload(cls, wl, **kw):
        return cls(wl.shape, wl.spacing, wl.dt, wl.shape_order, wl.center_order, wl.psatd_order, wl.dtype, **kw)

    def close(self):
        if self.ctx is not None and self.ctx.value:
            pic_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fields_from_workload(self, wl, device="cuda"):
        """Fields with the workload's initial E, B; rho_static from the ions; rho_old = rho^0."""
        import torch
        f = Fields(self.shape, self.dtype, device, averaged=bool(self.params.flags & PIC_AVERAGED))
        td = f.rho_old.dtype
        for d in range(3):
            f.E_stag[d].copy_(torch.from_numpy(wl.E[d]).to(td))
            f.B_stag[d].copy_(torch.from_numpy(wl.B[d]).to(td))
            if f.E_avg:  # the averaged fields of the first step: the initial fields
                f.E_avg[d].copy_(f.E_stag[d])
                f.B_avg[d].copy_(f.B_stag[d])
        return f

    def init_charge(self, f, electrons, ions):
        """rho_static <- deposit(ions); rho_old <- rho_static + deposit(electrons)."""
        if ions is not None:
            pic_deposit(self.ctx, [ions], f, PIC_DEP_RHO_ONLY)
            f.rho_static = f.rho_new.clone()
        pic_deposit(self.ctx, [electrons], f, PIC_DEP_RHO_ONLY)
        f.rho_old.copy_(f.rho_new)
