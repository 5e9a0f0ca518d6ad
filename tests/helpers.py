"""Error metrics shared by the parity tests.

Relative error is row-normwise per (point, component): the largest absolute
deviation over the row's functions divided by the row's largest reference
magnitude.  A plain elementwise relative error is undefined at the many
exact or near zeros of AOs, MOs and their derivatives.
"""
import numpy as np


def rownorm_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    num = np.max(np.abs(got - ref), axis=-1)
    den = np.maximum(np.max(np.abs(ref), axis=-1), 1e-300)
    return num / den


def component_errors(got, ref):
    """Max row-normwise error for value, gradient (3), Laplacian of arrays
    shaped [..., 5, n]."""
    e = rownorm_err(got, ref).reshape(-1, 5)
    return {"value": float(e[:, 0].max()), "gradient": float(e[:, 1:4].max()),
            "laplacian": float(e[:, 4].max())}


def grad_err(got, ref, ref_abs):
    """Elementwise error relative to the absolute sum of the terms."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(ref_abs, 1e-300)))
