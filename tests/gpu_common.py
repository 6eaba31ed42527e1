"""Shared helpers of the GPU parity tests (no method arithmetic: conversions and error norms)."""

import os
import sys

import numpy as np

EPS = {"f32": float(np.finfo(np.float32).eps), "f64": float(np.finfo(np.float64).eps)}


def banner(msg):
    """Name the case on stdout before any GPU work, so a failing run still says what ran."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_species(sp, shape, spacing):
    """Oracle species dict built from the device species (positions rounded as on the device)."""
    return {"pos": sp.positions(shape, spacing),
            "u": np.stack([np64(x) for x in sp.u], axis=1),
            "w": np64(sp.w), "q": sp.q, "m": sp.m}


def max_rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / scale) if scale > 0 else float(np.max(np.abs(got)))


def periodic_pos_err(pa, pb, lengths):
    d = np.abs(pa - pb)
    L = np.asarray(lengths)[None, :]
    d = np.minimum(d, L - d)
    return float(np.max(d)) if d.size else 0.0


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rounded(arrs, dtype):
    """The float64 arrays rounded to the run precision (what the device sees)."""
    npd = np.float32 if dtype == "f32" else np.float64
    return [np.asarray(a).astype(npd).astype(np.float64) for a in arrs]


def put(dst_list, arrs):
    """Copy host float64 arrays into device tensors (converted to their dtype)."""
    import torch
    for t, a in zip(dst_list, arrs):
        t.copy_(torch.from_numpy(np.asarray(a)).to(t.dtype))
