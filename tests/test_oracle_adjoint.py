"""The oracle's reverse mode of the field solve, pinned by the paper's time reversal of the
vacuum update (App. B): with no sources the update is a rotation per mode, so its
transpose is the update with -dt.  CPU only."""

import numpy as np

from oracle import adjoint
from oracle.step import Params, push_fields


def test_vacuum_transpose_is_time_reversed_update():
    rng = np.random.default_rng(5)
    shape = (8, 8, 8)
    p = Params(shape, (1.0, 1.0, 1.0), 0.7, 1, 8, 16)
    lam_E = [rng.standard_normal(shape) for _ in range(3)]
    lam_B = [rng.standard_normal(shape) for _ in range(3)]
    g = adjoint.push_fields_transpose(lam_E, lam_B, p)
    zero = np.zeros(shape)
    p_back = Params(shape, (1.0, 1.0, 1.0), -0.7, 1, 8, 16)
    E_back, B_back = push_fields(lam_E, lam_B, [zero, zero, zero], zero, zero, p_back)
    for d in range(3):
        np.testing.assert_allclose(g[d], E_back[d], atol=1e-12)
        np.testing.assert_allclose(g[3 + d], B_back[d], atol=1e-12)


def test_transpose_satisfies_the_dot_product_identity():
    rng = np.random.default_rng(6)
    shape = (8, 8, 8)
    p = Params(shape, (1.0, 1.0, 1.0), 0.5, 3, 8, 16)
    lam_E = [rng.standard_normal(shape) for _ in range(3)]
    lam_B = [rng.standard_normal(shape) for _ in range(3)]
    x = [rng.standard_normal(shape) for _ in range(11)]
    g = adjoint.push_fields_transpose(lam_E, lam_B, p)
    E, B = push_fields(x[0:3], x[3:6], x[6:9], x[9], x[10], p)
    lhs = sum(np.sum(lam_E[d] * E[d]) + np.sum(lam_B[d] * B[d]) for d in range(3))
    rhs = sum(np.sum(g[a] * x[a]) for a in range(11))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)
