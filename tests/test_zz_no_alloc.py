"""pic_deposit_noalloc (the deposition for callers that cannot allocate) against pic_deposit on the
same inputs, through the C ABI: two calls in a row on one context, the second with fewer
particles, each compared with pic_deposit to the deposition's FP32 bound; the call leaves the
device's free memory unchanged, where pic_deposit's first call on a species allocates its
scratch."""

import ctypes

import numpy as np
import pytest

from gpu_common import EPS, banner, max_rel, np64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2106_12919_amd import inputs  # noqa: E402
from paper_2106_12919_amd import lib as piclib  # noqa: E402


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _species(wl, n, dtype):
    sp = inputs.Species(cell=wl.electrons.cell[:n], off=wl.electrons.off[:n], u=wl.electrons.u[:n],
                        w=wl.electrons.w[:n], q=-1.0, m=1.0)
    return piclib.Species.from_host(sp, wl.shape, dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_deposit_matches_deposit(dtype):
    shape = (32, 24, 48)
    banner(f"pic_deposit_noalloc vs pic_deposit dtype={dtype} shape={shape}")
    wl = inputs.small(shape, ppc=8, shape_order=3, center_order=8, dtype=dtype, u_th=0.3, seed=141)
    n_all = wl.electrons.n
    tol = 1024 * EPS[dtype]
    ctx_a = piclib.Context.for_workload(wl)   # pic_deposit_noalloc only
    ctx_b = piclib.Context.for_workload(wl)   # pic_deposit
    # the HIP runtime's own lazy set-up of the kernels on their first launch is not the call's
    warm = _species(wl, 100, dtype)
    piclib.pic_deposit_noalloc(ctx_a.ctx, [warm], piclib.Fields(shape, dtype))
    piclib.pic_sync(ctx_a.ctx)
    for n in (n_all, n_all // 3 + 7):         # the second call smaller than the first
        sp = _species(wl, n, dtype)
        fa, fb = piclib.Fields(shape, dtype), piclib.Fields(shape, dtype)
        # stale values in the outputs: both entry points overwrite rho_new and J_nod
        for t in [fa.rho_new] + fa.J_nod:
            t.fill_(123.0)
        torch.cuda.synchronize()
        before = _free_bytes()
        piclib.pic_deposit_noalloc(ctx_a.ctx, [sp], fa)
        piclib.pic_sync(ctx_a.ctx)
        after = _free_bytes()
        assert after == before, (before, after)
        piclib.pic_deposit(ctx_b.ctx, [sp], fb)
        piclib.pic_sync(ctx_b.ctx)
        assert max_rel(np64(fa.rho_new), np64(fb.rho_new)) <= tol
        for d in range(3):
            assert max_rel(np64(fa.J_nod[d]), np64(fb.J_nod[d])) <= tol, d
    ctx_a.close()
    ctx_b.close()


def test_noalloc_deposit_rejects_oversized_species():
    banner("pic_deposit_noalloc size limit")
    shape = (16, 16, 16)
    ctx = piclib.Context(shape, (1.0, 1.0, 1.0), 0.5, 1, 4, 16, "f32")
    f = piclib.Fields(shape, "f32")
    n = 4194304 + 1
    sp = piclib.Species(torch.zeros(n, dtype=torch.int32, device="cuda"),
                        [torch.zeros(n, device="cuda") for _ in range(3)],
                        [torch.zeros(n, device="cuda") for _ in range(3)], torch.ones(n, device="cuda"), -1.0, 1.0)
    with pytest.raises(RuntimeError, match="particles in one species"):
        piclib.pic_deposit_noalloc(ctx.ctx, [sp], f)
    ctx.close()
