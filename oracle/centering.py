"""Finite-order centering between the nodal and the staggered (Yee) grid (oracle).

Test infrastructure only (see ``oracle/__init__``).

Staggered-to-nodal (Sec. 3, eq. ``staggered_finite_sum``; again in App. C):
    f_j = sum_{n=1}^{m} alpha^s_{m,n} (f_{j+n-1/2} + f_{j-n+1/2}) / 2.
Nodal-to-staggered: the paper prints only the staggered-to-nodal form.  Reading
used: the mirror image with the same coefficients,
    f_{j+1/2} = sum_{n=1}^{m} alpha^s_{m,n} (f_{j+n} + f_{j+1-n}) / 2,
which is the exact transpose of the staggered-to-nodal operator.

Storage convention: a staggered array along an axis holds f_{j+1/2} at index j.
Axes centred per component (App. A list of Yee positions): E^d and J^d along
their own axis d; B^d along the two axes other than d; rho is nodal on both
grids and is never centred.  Grids are periodic.
"""

import numpy as np

from .fornberg import alpha_staggered

STAGGERED_AXES = {
    "Ex": (0,), "Ey": (1,), "Ez": (2,),
    "Jx": (0,), "Jy": (1,), "Jz": (2,),
    "Bx": (1, 2), "By": (0, 2), "Bz": (0, 1),
}


def s2n_axis(f, axis, m):
    """Centre a staggered array to the nodes along ``axis`` at order 2m."""
    a = alpha_staggered(m)
    out = np.zeros_like(f, dtype=np.float64)
    for n in range(1, m + 1):
        plus = np.roll(f, -(n - 1), axis=axis)   # f_{j+n-1/2} is stored at index j+n-1
        minus = np.roll(f, n, axis=axis)         # f_{j-n+1/2} is stored at index j-n
        out += float(a[n - 1]) * 0.5 * (plus + minus)
    return out


def n2s_axis(f, axis, m):
    """Centre a nodal array to the cell centres along ``axis`` at order 2m (result at index j = position j+1/2)."""
    a = alpha_staggered(m)
    out = np.zeros_like(f, dtype=np.float64)
    for n in range(1, m + 1):
        plus = np.roll(f, -n, axis=axis)         # f_{j+n}
        minus = np.roll(f, n - 1, axis=axis)     # f_{j+1-n}
        out += float(a[n - 1]) * 0.5 * (plus + minus)
    return out


def s2n(name, f, m):
    """Staggered-to-nodal centering of component ``name`` (e.g. "Bx") along its staggered axes."""
    out = np.asarray(f, dtype=np.float64)
    for ax in STAGGERED_AXES[name]:
        out = s2n_axis(out, ax, m)
    return out


def n2s(name, f, m):
    """Nodal-to-staggered centering of component ``name`` along its staggered axes."""
    out = np.asarray(f, dtype=np.float64)
    for ax in STAGGERED_AXES[name]:
        out = n2s_axis(out, ax, m)
    return out
