"""FP64 CPU oracle (ctypes wrapper around liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  It shares no code with the GPU library.

All arrays are numpy complex128 in the canonical layouts
  gauge  U[Lt][Lz][Ly][Lx][mu][3][3]
  spinor psi[(nrhs,)][Lt][Lz][Ly][Lx][4][3]
and the lattice extents (Lx, Ly, Lz, Lt) are read off the gauge field.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import dense  # noqa: F401  (brute-force dense path, re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_hop.argtypes = [_ip, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_hop_sites.argtypes = [_ip, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_long),
                                     ctypes.c_long, _dp, ctypes.c_int]
    lib.oracle_apply_M.argtypes = [_ip, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_apply_M_sites.argtypes = [_ip, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_long), ctypes.c_long, _dp,
                                         ctypes.c_int]
    lib.oracle_apply_schur.argtypes = [_ip, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp,
                                       ctypes.c_int]
    lib.oracle_clover.argtypes = [_ip, ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.oracle_field_strength.argtypes = [_ip, _dp, ctypes.c_int, ctypes.c_int, _dp]
    lib.oracle_site_inverse.argtypes = [ctypes.c_long, _dp, _dp]
    lib.oracle_site_inverse.restype = ctypes.c_int
    lib.oracle_cg.argtypes = [_ip, ctypes.c_double, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_force.argtypes = [_ip, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_plaquette.argtypes = [_ip, _dp]
    lib.oracle_plaquette.restype = ctypes.c_double
    lib.oracle_gamma.argtypes = [ctypes.c_int, _dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _arr(a):
    if hasattr(a, "detach"):  # torch tensor on the CPU
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _dims(U):
    lt, lz, ly, lx = U.shape[:4]
    if U.shape[4:] != (4, 3, 3):
        raise ValueError(f"gauge field must be (Lt,Lz,Ly,Lx,4,3,3), got {U.shape}")
    return (ctypes.c_int * 4)(lx, ly, lz, lt)


def _bc(bc):
    b = np.ascontiguousarray(np.asarray(bc, dtype=np.float64).reshape(8))
    return b


def _per_rhs(fn, psi, site_shape):
    """Apply fn to each right-hand side of psi (leading axis optional)."""
    if psi.shape == site_shape:
        return fn(psi)
    return np.stack([fn(np.ascontiguousarray(p)) for p in psi])


def num_threads() -> int:
    return _load().oracle_num_threads()


def gamma(mu: int) -> np.ndarray:
    out = np.zeros(32)
    _load().oracle_gamma(mu, out.ctypes.data_as(_dp))
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def hop(U, psi, bc, dagger=False):
    """D psi (dagger: D^H psi = g5 D g5 psi)."""
    U, psi, b = _arr(U), _arr(psi), _bc(bc)
    L = _dims(U)
    lib = _load()

    def one(p):
        out = np.empty_like(p)
        lib.oracle_hop(L, _ptr(b), _ptr(U), _ptr(p), _ptr(out), int(dagger))
        return out
    return _per_rhs(one, psi, U.shape[:4] + (4, 3))


def hop_sites(U, psi, bc, sites, dagger=False):
    """(D psi) at the given lexicographic site indices only, shape (n, 4, 3)."""
    U, psi, b = _arr(U), _arr(psi), _bc(bc)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((len(s), 4, 3), dtype=np.complex128)
    _load().oracle_hop_sites(_dims(U), _ptr(b), _ptr(U), _ptr(psi),
                             s.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(s), _ptr(out),
                             int(dagger))
    return out


def apply_M_sites(U, psi, kappa, bc, sites, csw=0.0, dagger=False):
    """(M psi) at the given lexicographic sites only (clover built locally), shape (n,4,3)."""
    U, psi, b = _arr(U), _arr(psi), _bc(bc)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((len(s), 4, 3), dtype=np.complex128)
    _load().oracle_apply_M_sites(_dims(U), kappa, csw, _ptr(b), _ptr(U), _ptr(psi),
                                 s.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(s),
                                 _ptr(out), int(dagger))
    return out


def apply_M(U, psi, kappa, bc, clover=None, dagger=False):
    """M psi = A psi - kappa D psi (A = 1 unless a clover field is given)."""
    U, psi, b = _arr(U), _arr(psi), _bc(bc)
    A = None if clover is None else _arr(clover)
    L = _dims(U)
    lib = _load()

    def one(p):
        out = np.empty_like(p)
        lib.oracle_apply_M(L, kappa, _ptr(b), _ptr(U), _ptr(A), _ptr(p), _ptr(out), int(dagger))
        return out
    return _per_rhs(one, psi, U.shape[:4] + (4, 3))


def apply_schur(U, psi, kappa, bc, clover=None, clover_inv=None, dagger=False):
    """Even-site Schur complement S = A_ee - kappa^2 D_eo A_oo^-1 D_oe on full-lattice arrays."""
    U, psi, b = _arr(U), _arr(psi), _bc(bc)
    A = None if clover is None else _arr(clover)
    Ai = None if clover_inv is None else _arr(clover_inv)
    if (A is None) != (Ai is None):
        raise ValueError("clover and clover_inv go together")
    L = _dims(U)
    lib = _load()

    def one(p):
        out = np.empty_like(p)
        lib.oracle_apply_schur(L, kappa, _ptr(b), _ptr(U), _ptr(A), _ptr(Ai), _ptr(p), _ptr(out),
                               int(dagger))
        return out
    return _per_rhs(one, psi, U.shape[:4] + (4, 3))


def clover(U, kappa, csw):
    """Per-site 12x12 clover matrix A, shape (Lt,Lz,Ly,Lx,12,12)."""
    U = _arr(U)
    A = np.empty(U.shape[:4] + (12, 12), dtype=np.complex128)
    _load().oracle_clover(_dims(U), kappa, csw, _ptr(U), _ptr(A))
    return A


def field_strength(U, mu, nu):
    U = _arr(U)
    F = np.empty(U.shape[:4] + (3, 3), dtype=np.complex128)
    _load().oracle_field_strength(_dims(U), _ptr(U), mu, nu, _ptr(F))
    return F


def site_inverse(A):
    A = _arr(A)
    B = np.empty_like(A)
    n = A.size // 144
    if _load().oracle_site_inverse(n, _ptr(A), _ptr(B)) != 0:
        raise ZeroDivisionError("singular site matrix")
    return B


def cg(U, b, kappa, bc, system=0, tol=1e-10, max_iter=10000, fixed_iters=0, clover=None,
       clover_inv=None):
    """CG on M^H M (system 0) or the even-site S^H S (system 1), x0 = 0.

    Returns (x, iterations, true_relative_residual); iterations is -1 when
    max_iter is hit unconverged.  Multiple right-hand sides run one by one.
    """
    U, b, bcv = _arr(U), _arr(b), _bc(bc)
    A = None if clover is None else _arr(clover)
    Ai = None if clover_inv is None else _arr(clover_inv)
    if system == 1 and A is not None and Ai is None:
        Ai = site_inverse(A)
    L = _dims(U)
    lib = _load()
    site_shape = U.shape[:4] + (4, 3)
    single = b.shape == site_shape
    bs = b[None] if single else b
    xs, its, res = [], [], []
    for bb in bs:
        bb = np.ascontiguousarray(bb)
        x = np.empty_like(bb)
        r = ctypes.c_double(0.0)
        it = lib.oracle_cg(L, kappa, _ptr(bcv), _ptr(U), _ptr(A), _ptr(Ai), int(system), _ptr(bb),
                           _ptr(x), tol, int(max_iter), int(fixed_iters), ctypes.byref(r))
        xs.append(x)
        its.append(it)
        res.append(r.value)
    if single:
        return xs[0], its[0], res[0]
    return np.stack(xs), its, res


def force(U, X, Y, kappa, bc, mode=0):
    """Fermion force per link: mode 0 = dS/dReU + i dS/dImU, mode 1 = traceless Hermitian F."""
    U, X, Y, b = _arr(U), _arr(X), _arr(Y), _bc(bc)
    F = np.empty_like(U)
    _load().oracle_force(_dims(U), kappa, _ptr(b), _ptr(U), _ptr(X), _ptr(Y), _ptr(F), int(mode))
    return F


def plaquette(U):
    U = _arr(U)
    return _load().oracle_plaquette(_dims(U), _ptr(U))


def parity_mask(dims):
    """Boolean (Lt,Lz,Ly,Lx) array, True on even sites."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2) == 0
