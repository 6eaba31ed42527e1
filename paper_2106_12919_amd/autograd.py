"""Reverse mode of the field solve and of the centering, as torch.autograd Functions.

Both are linear maps whose transposes the library computes (``psatd_push_fields_adjoint``,
and ``pic_center`` with the opposite direction), so a loss can be differentiated through
them with torch's autograd.  Every computation runs in libpic's HIP kernels; this module
only moves tensors in and out of a ``Fields`` workspace.
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
