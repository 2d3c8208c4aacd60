"""Small helpers shared by the tests (no operator arithmetic)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def g5(psi):
    """gamma5 = diag(1,1,-1,-1) in the chiral basis (spin axis is -2)."""
    out = np.array(psi, copy=True)
    out[..., 2:, :] *= -1
    return out


def dims_of(U):
    lt, lz, ly, lx = U.shape[:4]
    return (lx, ly, lz, lt)
