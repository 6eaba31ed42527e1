"""Reverse mode of the field solve (oracle).

Test infrastructure only (see ``oracle/__init__``).

The field solve of one step, ``step.push_fields`` (Sec. 4.2), is linear in
(E^n, B^n, J^{n+1/2}, rho^n, rho^{n+1}).  Its transpose is built here by brute force:
column c of the Jacobian is the response to the unit input c, and the adjoint input
lambda contracts it to one gradient entry.  Obviously correct and slow (tiny grids).
"""

import numpy as np

from .step import push_fields


def push_fields_transpose(lam_E, lam_B, p):
    """dL/d(E, B, J, rho_old, rho_new) for dL/dE' = lam_E, dL/dB' = lam_B (lists of 3 arrays).

    Returns a list of 11 arrays: E (3), B (3), J (3), rho_old, rho_new."""
    shape = p.shape
    grads = [np.zeros(shape) for _ in range(11)]
    for a in range(11):
        for idx in np.ndindex(*shape):
            x = [np.zeros(shape) for _ in range(11)]
            x[a][idx] = 1.0
            E, B = push_fields(x[0:3], x[3:6], x[6:9], x[9], x[10], p)
            grads[a][idx] = sum(float(np.sum(lam_E[d] * E[d]) + np.sum(lam_B[d] * B[d])) for d in range(3))
    return grads
