"""Reverse mode of the hybrid PIC cycle as torch.autograd Functions.

* ``PsatdPushFields`` and ``Center``: the field solve and the centering, linear maps whose
  transposes the library computes (``psatd_push_fields_adjoint``, and ``pic_center`` with the
  opposite direction).
* ``PicSteps``: nsteps whole cycles (``pic_step`` with the caller's particle order kept) with
  gradients with respect to the initial fields, charge density, particle offsets and momenta,
  by ``pic_step_adjoint`` one step at a time, backwards, from states recomputed out of
  checkpoints kept every ``checkpoint_every`` steps (every step, with nothing recomputed, when
  ``checkpoint_interval`` finds that the states fit in the memory given to them).

Every computation runs in libpic's HIP kernels; this module only moves tensors in and out
of the library's workspaces and keeps the checkpoints.
"""

import torch

from . import lib as piclib


def _fields(pic):
    return piclib.Fields(pic.shape, pic.dtype)


def _put(dst, src):
    for d in range(3):
        dst[d].copy_(src[d])


class PsatdPushFields(torch.autograd.Function):
    """(E^n, B^n, J^{n+1/2}, rho^n, rho^{n+1}) -> (E^{n+1}, B^{n+1}) on the staggered grid.

    E, B, J: tensors (3, nx, ny, nz) of the context's dtype on its device; rho: (nx, ny, nz).
    ``pic`` is a ``lib.Context``."""

    @staticmethod
    def forward(ctx, pic, E, B, J, rho_old, rho_new):
        f = _fields(pic)
        _put(f.E_stag, E)
        _put(f.B_stag, B)
        _put(f.J_stag, J)
        f.rho_old.copy_(rho_old)
        f.rho_new.copy_(rho_new)
        piclib.psatd_push_fields(pic.ctx, f)
        ctx.pic = pic
        return torch.stack(f.E_stag), torch.stack(f.B_stag)

    @staticmethod
    def backward(ctx, gE, gB):
        pic = ctx.pic
        f = _fields(pic)
        _put(f.E_stag, gE.contiguous())
        _put(f.B_stag, gB.contiguous())
        piclib.psatd_push_fields_adjoint(pic.ctx, f)
        return None, torch.stack(f.E_stag), torch.stack(f.B_stag), torch.stack(f.J_stag), f.rho_old, f.rho_new


_CENTER_IO = {  # (dir, what) -> (input array name, output array name)
    (piclib.PIC_N2S, piclib.PIC_J): ("J_nod", "J_stag"),
    (piclib.PIC_S2N, piclib.PIC_J): ("J_stag", "J_nod"),
    (piclib.PIC_S2N, piclib.PIC_E): ("E_stag", "E_nod"),
    (piclib.PIC_N2S, piclib.PIC_E): ("E_nod", "E_stag"),
    (piclib.PIC_S2N, piclib.PIC_B): ("B_stag", "B_nod"),
    (piclib.PIC_N2S, piclib.PIC_B): ("B_nod", "B_stag"),
}


def _center(pic, direction, what, x):
    src, dst = _CENTER_IO[(direction, what)]
    f = _fields(pic)
    _put(getattr(f, src), x)
    piclib.pic_center(pic.ctx, direction, what, f)
    return torch.stack(getattr(f, dst))


class Center(torch.autograd.Function):
    """Finite-order centering of a 3-component field, ``direction`` / ``what`` as in pic_center;
    its backward is the transposed centering (the opposite direction)."""

    @staticmethod
    def forward(ctx, pic, direction, what, x):
        ctx.pic, ctx.direction, ctx.what = pic, direction, what
        return _center(pic, direction, what, x)

    @staticmethod
    def backward(ctx, g):
        back = piclib.PIC_S2N if ctx.direction == piclib.PIC_N2S else piclib.PIC_N2S
        return None, None, None, _center(ctx.pic, back, ctx.what, g.contiguous())


class DifferentiableRun:
    """Fixed data of a differentiable run: a ``lib.Context`` created with PIC_KEEP_ORDER in its
    flags, one mobile species' charge and mass, an optional static background charge, the
    number of steps and the checkpoint interval."""

    def __init__(self, pic, q, m, nsteps, checkpoint_every=10, rho_static=None):
        if not (pic.params.flags & piclib.PIC_KEEP_ORDER):
            raise ValueError("the context needs PIC_KEEP_ORDER (particles followed by index across steps)")
        if nsteps < 1 or checkpoint_every < 1:
            raise ValueError("nsteps and checkpoint_every must be >= 1")
        self.pic, self.q, self.m = pic, float(q), float(m)
        self.nsteps, self.every = int(nsteps), int(checkpoint_every)
        self.rho_static = rho_static
        self.work = _fields(pic)  # E_nod, B_nod, J, rho_new workspace of the forward steps
        self.work.rho_static = rho_static


class _State:
    """E, B (Yee), rho^n and one species' cell, offsets, momenta, held in three contiguous
    buffers (fields (7, nx, ny, nz); cell (Np,); off and u as rows of one (6, Np_pad) float
    buffer whose rows start 256-byte aligned), so that a copy of the state is three copies."""

    def __init__(self, fbuf, cell, pbuf, n):
        self.fbuf, self.cell, self.pbuf, self.n = fbuf, cell, pbuf, n
        self.E = [fbuf[d] for d in range(3)]
        self.B = [fbuf[3 + d] for d in range(3)]
        self.rho = fbuf[6]
        self.off = [pbuf[d, :n] for d in range(3)]
        self.u = [pbuf[3 + d, :n] for d in range(3)]

    @classmethod
    def of(cls, E, B, rho, cell, off, u):
        fbuf = torch.stack([*(E[d] for d in range(3)), *(B[d] for d in range(3)), rho]).detach().contiguous()
        n = int(cell.numel())
        row = -(-n // 64) * 64  # 64 elements: at least 256 bytes per row start
        pbuf = torch.zeros((6, row), dtype=fbuf.dtype, device=fbuf.device)
        for d in range(3):
            pbuf[d, :n].copy_(off[d].detach())
            pbuf[3 + d, :n].copy_(u[d].detach())
        return cls(fbuf, cell.detach().clone().contiguous(), pbuf, n)

    def clone(self):
        return _State(self.fbuf.clone(), self.cell.clone(), self.pbuf.clone(), self.n)

    def fields(self, run):
        f = run.work
        f.E_stag, f.B_stag, f.rho_old = self.E, self.B, self.rho
        return f

    def species(self, run, w):
        return piclib.Species(self.cell, self.off, self.u, w, run.q, run.m)

    def step(self, run, w, n):
        piclib.pic_step(run.pic.ctx, self.fields(run), [self.species(run, w)], n)


def state_bytes(pic, n_particles):
    """Device bytes of one stored state of a run (the _State buffers): E, B, rho and one species'
    cell, offsets and momenta."""
    elem = 4 if pic.dtype == "f32" else 8
    nx, ny, nz = pic.shape
    row = -(-int(n_particles) // 64) * 64
    return 7 * nx * ny * nz * elem + 4 * int(n_particles) + 6 * row * elem


def checkpoint_interval(pic, n_particles, nsteps, budget_bytes):
    """The smallest checkpoint interval k whose states fit in ``budget_bytes``: ceil(nsteps / k)
    checkpoints, plus, when k > 1, the k states of one segment recomputed in the backward pass and
    its working copy.  k = 1 stores every step's state, and the backward pass then recomputes
    nothing.  When no interval fits, the one that holds the fewest states."""
    s = state_bytes(pic, n_particles)
    n = int(nsteps)

    def held(k):
        return -(-n // k) + (k + 1 if k > 1 else 0)

    for k in range(1, n + 1):
        if held(k) * s <= budget_bytes:
            return k
    return min(range(1, n + 1), key=held)  # none fits: the fewest states held


def _zeros_or(g, like):
    return torch.zeros_like(like) if g is None else g.contiguous()


class PicSteps(torch.autograd.Function):
    """run.nsteps hybrid cycles: (E, B, rho, off, u) at step 0 -> the same at step nsteps.

    E, B: (3, nx, ny, nz) on the Yee grid; rho: (nx, ny, nz) = rho^0 (rho_old); cell: (Np,) int32;
    w: (Np,) weights; off, u: (3, Np).  Returns (E, B, rho, cell, off, u) after the run, the
    particles in the input order (cell is not differentiable).  The backward pass recomputes
    each checkpoint segment forward, keeping its states, and applies pic_step_adjoint from the
    last step of the segment to the first."""

    @staticmethod
    def forward(ctx, run, cell, w, E, B, rho, off, u):
        st = _State.of(E, B, rho, cell, off, u)
        w = w.detach().contiguous()
        checkpoints = [st.clone()]
        n = 0
        while n < run.nsteps:
            k = min(run.every, run.nsteps - n)
            st.step(run, w, k)
            n += k
            if n < run.nsteps:
                checkpoints.append(st.clone())
        ctx.run, ctx.w, ctx.checkpoints = run, w, checkpoints
        out_cell = st.cell.clone()
        ctx.mark_non_differentiable(out_cell)
        return (torch.stack(st.E), torch.stack(st.B), st.rho.clone(), out_cell, torch.stack(st.off),
                torch.stack(st.u))

    @staticmethod
    def backward(ctx, gE, gB, grho, gcell, goff, gu):
        run, w = ctx.run, ctx.w
        ref = ctx.checkpoints[0]
        adj = _fields(run.pic)
        gE = _zeros_or(gE, torch.stack(ref.E))
        gB = _zeros_or(gB, torch.stack(ref.B))
        for d in range(3):
            adj.E_stag[d].copy_(gE[d])
            adj.B_stag[d].copy_(gB[d])
        adj.rho_new.copy_(_zeros_or(grho, ref.rho))
        goff = _zeros_or(goff, torch.stack(ref.off))
        gu = _zeros_or(gu, torch.stack(ref.u))
        asp = piclib.SpeciesAdjoint([goff[d].clone() for d in range(3)], [gu[d].clone() for d in range(3)])
        for seg in reversed(range(len(ctx.checkpoints))):
            n0 = seg * run.every
            k = min(run.every, run.nsteps - n0)
            if k == 1:  # pic_step_adjoint only reads the state: the checkpoint itself serves
                states = [ctx.checkpoints[seg]]
            else:
                st = ctx.checkpoints[seg].clone()
                states = [st.clone()]
                for _ in range(k - 1):
                    st.step(run, w, 1)
                    states.append(st.clone())
            ctx.checkpoints[seg] = None  # not needed again: free it for the segments before
            for sj in reversed(states):
                piclib.pic_step_adjoint(run.pic.ctx, sj.fields(run), [sj.species(run, w)], adj, [asp])
                adj.rho_old, adj.rho_new = adj.rho_new, adj.rho_old  # dL/drho^n carries to the step before
        ctx.checkpoints = None
        return (None, None, None, torch.stack(adj.E_stag), torch.stack(adj.B_stag), adj.rho_new.clone(),
                torch.stack(asp.off), torch.stack(asp.u))
