"""Small helpers shared by the tests (no operator arithmetic)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def site_err(a, b, block=12):
    """Largest per-site error: max over sites s of |a_s - b_s| / max_s |b_s|, where a site
    is a trailing block of `block` entries (a spinor's (4, 3) by default; 36 for the
    (4, 3, 3) links of a site).  Unlike the norm-wise rel(), one bad site among millions
    cannot hide in the average."""
    a = np.asarray(a).reshape(-1, block)
    b = np.asarray(b).reshape(-1, block)
    scale = max(float(np.max(np.linalg.norm(b, axis=1))), 1e-300)
    return float(np.max(np.linalg.norm(a - b, axis=1)) / scale)


def assert_close(got, ref, tol, what="", block=12):
    """Norm-wise and per-site agreement to tol."""
    r, s = rel(got, ref), site_err(got, ref, block)
    assert r <= tol and s <= tol, (what, r, s, tol)


def g5(psi):
    """gamma5 = diag(1,1,-1,-1) in the chiral basis (spin axis is -2)."""
    out = np.array(psi, copy=True)
    out[..., 2:, :] *= -1
    return out


def dims_of(U):
    lt, lz, ly, lx = U.shape[:4]
    return (lx, ly, lz, lt)
