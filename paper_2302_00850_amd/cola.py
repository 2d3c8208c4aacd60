"""ctypes binding of libcola.so (include/cola.h).

The module-level functions carry the C names and only marshal arguments:
device buffers are passed as integer addresses (``tensor.data_ptr()``), the
stream as ``torch.cuda.current_stream().cuda_stream``.  Every computation runs
in the HIP library; there is no fallback path.  ``Lattice`` is a thin
convenience layer over the same calls, with torch tensors supplying device
memory; ``PseudofermionAction`` exposes the fermion action and its force to
torch autograd.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcola.so")

# ---- constants mirrored from include/cola.h
COLA_OK, COLA_EINVAL, COLA_EHIP, COLA_ENOMEM, COLA_ESTATE = 0, -1, -2, -3, -4
COLA_NOT_CONVERGED, COLA_BREAKDOWN = 1, 2
COLA_FP64, COLA_FP64_12, COLA_FP32, COLA_FP16 = 0, 1, 2, 3
(COLA_OP_HOP, COLA_OP_HOP_DAG, COLA_OP_M, COLA_OP_MDAG, COLA_OP_MDAGM, COLA_OP_SCHUR,
 COLA_OP_SCHUR_DAG, COLA_OP_SCHUR_DAGSCHUR) = range(8)
COLA_SYS_MDAGM, COLA_SYS_SCHUR, COLA_SYS_PROPAGATOR = 0, 1, 2
COLA_CG_FP64, COLA_CG_FP32_RELIABLE, COLA_CG_FP16_DEFECT, COLA_CG_FP32_DEFECT = 0, 1, 2, 3
COLA_FLAG_TIMING = 1
COLA_FORCE_GRAD, COLA_FORCE_LIE = 0, 1
(COLA_HOP_PLAIN, COLA_HOP_XPAY, COLA_HOP_CLOV, COLA_HOP_CLOV_XPAY, COLA_HOP_XPAY_CLOV,
 COLA_HOP_XPAY_CG, COLA_HOP_CLOV_XPAY_CG) = range(7)
MAX_RHS = 16


class ColaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cola error {code}: {msg}")
        self.code = code


class CgParams(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("scheme", ctypes.c_int), ("block", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("reliable_interval", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("use_x0", ctypes.c_int), ("check_interval", ctypes.c_int)]


class CgResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("outer_cycles", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("true_rel_residual", ctypes.POINTER(ctypes.c_double)),
                ("seconds", ctypes.c_double)]


class EigParams(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("tol", ctypes.c_double),
                ("inner_reduction", ctypes.c_double), ("inner_max", ctypes.c_int),
                ("max_sweeps", ctypes.c_int)]


class EigResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("applications", ctypes.c_int),
                ("eigenvalues", ctypes.POINTER(ctypes.c_double)),
                ("residuals", ctypes.POINTER(ctypes.c_double)), ("seconds", ctypes.c_double)]


class HmcParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("nsteps", ctypes.c_int),
                ("cg_tol", ctypes.c_double), ("cg_max_iter", ctypes.c_int), ("eo", ctypes.c_int),
                ("integrator", ctypes.c_int), ("n_gauge", ctypes.c_int),
                ("cg_scheme", ctypes.c_int)]


class HmcResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("dH", ctypes.c_double), ("kinetic0", ctypes.c_double),
                ("kinetic1", ctypes.c_double), ("gauge0", ctypes.c_double),
                ("gauge1", ctypes.c_double), ("fermion0", ctypes.c_double),
                ("fermion1", ctypes.c_double), ("cg_iterations", ctypes.c_int),
                ("seconds", ctypes.c_double)]


HOP_KINDS = 8


class Stats(ctypes.Structure):
    _fields_ = [("hop_launches", ctypes.c_longlong * 4), ("hop_seconds", ctypes.c_double * 4),
                ("hop_bytes", ctypes.c_double * 4), ("hop_flops", ctypes.c_double * 4),
                ("kind_launches", (ctypes.c_longlong * HOP_KINDS) * 4),
                ("kind_seconds", (ctypes.c_double * HOP_KINDS) * 4),
                ("kind_bytes", (ctypes.c_double * HOP_KINDS) * 4)]


EXPORTS = ["cola_abi_version", "cola_create", "cola_destroy", "cola_last_error", "cola_set_gauge",
           "cola_gauge_is_su3", "cola_field_bytes", "cola_pack_spinor", "cola_unpack_spinor",
           "cola_dslash_apply", "cola_cg_solve", "cola_fermion_force", "cola_get_stats",
           "cola_reset_stats", "cola_set_tuning", "cola_tune_dump", "cola_gauge_force",
           "cola_gauge_action", "cola_link_update", "cola_momentum_update",
           "cola_hmc_trajectory", "cola_cg_multishift", "cola_fermion_action",
           "cola_dslash_apply_noalloc", "cola_eigensolve", "cola_cg_deflated",
           "cola_ape_smear", "cola_set_fat_gauge", "cola_tune_load", "cola_tune_save"]

_lib = None
_vp = ctypes.c_void_p


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2302_00850_amd.build`")
    lib = ctypes.CDLL(path)
    lib.cola_abi_version.restype = ctypes.c_int
    lib.cola_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_uint]
    lib.cola_destroy.argtypes = [_vp]
    lib.cola_last_error.argtypes = [_vp]
    lib.cola_last_error.restype = ctypes.c_char_p
    lib.cola_set_gauge.argtypes = [_vp, _vp, _vp]
    lib.cola_gauge_is_su3.argtypes = [_vp]
    lib.cola_field_bytes.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.cola_field_bytes.restype = ctypes.c_size_t
    lib.cola_pack_spinor.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]
    lib.cola_unpack_spinor.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]
    lib.cola_dslash_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _vp]
    lib.cola_dslash_apply_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, _vp]
    lib.cola_cg_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(CgParams),
                                  ctypes.POINTER(CgResult), _vp]
    lib.cola_fermion_force.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]
    lib.cola_fermion_action.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int), _vp]
    lib.cola_get_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
    lib.cola_reset_stats.argtypes = [_vp]
    lib.cola_set_tuning.argtypes = [_vp, ctypes.c_int]
    lib.cola_tune_dump.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.cola_tune_dump.restype = ctypes.c_size_t
    lib.cola_tune_load.argtypes = [_vp, ctypes.c_char_p]
    lib.cola_tune_save.argtypes = [_vp, ctypes.c_char_p]
    lib.cola_cg_multishift.argtypes = [_vp, _vp, _vp, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(CgParams),
                                       ctypes.POINTER(CgResult), _vp]
    lib.cola_eigensolve.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(EigParams),
                                    ctypes.POINTER(EigResult), _vp]
    lib.cola_cg_deflated.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                     ctypes.POINTER(CgParams), ctypes.POINTER(CgResult), _vp]
    lib.cola_ape_smear.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp]
    lib.cola_set_fat_gauge.argtypes = [_vp, _vp, _vp]
    lib.cola_gauge_force.argtypes = [_vp, _vp, _vp, ctypes.c_double, _vp]
    lib.cola_gauge_action.argtypes = [_vp, _vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                      _vp]
    lib.cola_link_update.argtypes = [_vp, _vp, _vp, ctypes.c_double, _vp]
    lib.cola_momentum_update.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, _vp]
    lib.cola_hmc_trajectory.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(HmcParams),
                                        ctypes.POINTER(HmcResult), _vp]
    _lib = lib
    return lib


def _check(h, rc):
    if rc < 0:
        msg = load().cola_last_error(h).decode() if h else ""
        raise ColaError(rc, msg)
    return rc


# ------------------------------------------------------------- C-named calls

def cola_abi_version() -> int:
    return load().cola_abi_version()


def cola_create(dims, kappa, bc_phase, csw=0.0, flags=0):
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    ph = (ctypes.c_double * 8)(*np.asarray(bc_phase, dtype=np.float64).reshape(8))
    h = _vp()
    rc = load().cola_create(ctypes.byref(h), d, float(kappa), ph, float(csw), int(flags))
    if rc != COLA_OK:
        raise ColaError(rc, "cola_create failed (dims must be even and >= 2)")
    return h


def cola_destroy(h):
    return load().cola_destroy(h)


def cola_last_error(h) -> str:
    return load().cola_last_error(h).decode()


def cola_set_gauge(h, U_ptr, stream=None):
    return _check(h, load().cola_set_gauge(h, U_ptr, stream))


def cola_gauge_is_su3(h) -> int:
    return load().cola_gauge_is_su3(h)


def cola_field_bytes(h, prec, nrhs, parity) -> int:
    return load().cola_field_bytes(h, prec, nrhs, parity)


def cola_pack_spinor(h, dst, src, prec, nrhs, parity, stream=None):
    return _check(h, load().cola_pack_spinor(h, dst, src, prec, nrhs, parity, stream))


def cola_unpack_spinor(h, dst, src, prec, nrhs, parity, stream=None):
    return _check(h, load().cola_unpack_spinor(h, dst, src, prec, nrhs, parity, stream))


def cola_dslash_apply(h, out, inp, op, parity, prec, nrhs, stream=None):
    return _check(h, load().cola_dslash_apply(h, out, inp, op, parity, prec, nrhs, stream))


def cola_dslash_apply_noalloc(h, out, inp, op, parity, prec, nrhs, stream=None):
    return _check(h, load().cola_dslash_apply_noalloc(h, out, inp, op, parity, prec, nrhs,
                                                      stream))


def cola_cg_solve(h, x, b, nrhs, params: CgParams, result: CgResult, stream=None):
    return _check(h, load().cola_cg_solve(h, x, b, nrhs, ctypes.byref(params),
                                          ctypes.byref(result), stream))


def cola_fermion_force(h, F, X, Y, mode, stream=None):
    return _check(h, load().cola_fermion_force(h, F, X, Y, mode, stream))


def cola_fermion_action(h, phi, X, Y, tol, stream=None):
    """(status, S, iterations) of S = Re <phi, X>, X = (M^H M)^{-1} phi, Y = M X."""
    S = ctypes.c_double()
    it = ctypes.c_int()
    rc = _check(h, load().cola_fermion_action(h, phi, X, Y, float(tol), ctypes.byref(S),
                                              ctypes.byref(it), stream))
    return rc, S.value, it.value


def cola_cg_multishift(h, x, b, nshift, shifts, params: CgParams, result: CgResult,
                       stream=None):
    sh = (ctypes.c_double * nshift)(*[float(v) for v in shifts])
    return _check(h, load().cola_cg_multishift(h, x, b, int(nshift), sh, ctypes.byref(params),
                                               ctypes.byref(result), stream))


def cola_eigensolve(h, X, n, params: EigParams, result: EigResult, stream=None):
    return _check(h, load().cola_eigensolve(h, X, n, ctypes.byref(params), ctypes.byref(result),
                                            stream))


def cola_cg_deflated(h, x, b, nrhs, X, lam, n, params: CgParams, result: CgResult, stream=None):
    lam_arr = (ctypes.c_double * n)(*lam)
    return _check(h, load().cola_cg_deflated(h, x, b, nrhs, X, lam_arr, n, ctypes.byref(params),
                                             ctypes.byref(result), stream))


def cola_ape_smear(h, F, U, alpha, nsweeps, stream=None):
    return _check(h, load().cola_ape_smear(h, F, U, alpha, nsweeps, stream))


def cola_set_fat_gauge(h, F, stream=None):
    return _check(h, load().cola_set_fat_gauge(h, F, stream))


def cola_gauge_force(h, F, U, beta, stream=None):
    return _check(h, load().cola_gauge_force(h, F, U, float(beta), stream))


def cola_gauge_action(h, U, beta, stream=None) -> float:
    S = ctypes.c_double()
    _check(h, load().cola_gauge_action(h, U, float(beta), ctypes.byref(S), stream))
    return S.value


def cola_link_update(h, U, P, eps, stream=None):
    return _check(h, load().cola_link_update(h, U, P, float(eps), stream))


def cola_momentum_update(h, P, F1, F2, eps, stream=None):
    return _check(h, load().cola_momentum_update(h, P, F1, F2, float(eps), stream))


def cola_hmc_trajectory(h, U, P, phi, params: HmcParams, result: HmcResult, stream=None):
    return _check(h, load().cola_hmc_trajectory(h, U, P, phi, ctypes.byref(params),
                                                 ctypes.byref(result), stream))


def cola_get_stats(h) -> Stats:
    s = Stats()
    _check(h, load().cola_get_stats(h, ctypes.byref(s)))
    return s


def cola_reset_stats(h):
    return _check(h, load().cola_reset_stats(h))


def cola_set_tuning(h, mode):
    return _check(h, load().cola_set_tuning(h, mode))


def cola_tune_load(h, path=None) -> int:
    return _check(h, load().cola_tune_load(h, path.encode() if path else None))


def cola_tune_save(h, path=None) -> int:
    return _check(h, load().cola_tune_save(h, path.encode() if path else None))


def cola_tune_dump(h) -> str:
    n = load().cola_tune_dump(h, None, 0)
    buf = ctypes.create_string_buffer(n)
    load().cola_tune_dump(h, buf, n)
    return buf.value.decode()


# ------------------------------------------------------------- convenience

def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return t.data_ptr()


class Lattice:
    """A handle bound to a lattice shape, kappa, boundary phases and c_sw."""

    def __init__(self, dims, kappa, bc_phase, csw=0.0, flags=0):
        self.dims = tuple(int(v) for v in dims)
        self.kappa = float(kappa)
        self.bc_phase = np.asarray(bc_phase, dtype=np.float64).reshape(4, 2)
        self.csw = float(csw)
        self.h = cola_create(self.dims, self.kappa, self.bc_phase, self.csw, flags)
        lx, ly, lz, lt = self.dims
        self.site_shape = (lt, lz, ly, lx)

    def close(self):
        if self.h:
            cola_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # fields
    def set_gauge(self, U: torch.Tensor):
        if U.dtype != torch.complex128 or tuple(U.shape) != self.site_shape + (4, 3, 3):
            raise ValueError("gauge field must be complex128 (Lt,Lz,Ly,Lx,4,3,3)")
        cola_set_gauge(self.h, _ptr(U), _stream())

    @property
    def gauge_is_su3(self) -> bool:
        return bool(cola_gauge_is_su3(self.h))

    def empty_packed(self, prec, nrhs=1, parity=-1) -> torch.Tensor:
        n = cola_field_bytes(self.h, prec, nrhs, parity)
        if n == 0:
            raise ValueError("bad precision / nrhs / parity")
        return torch.zeros(n, dtype=torch.uint8, device="cuda")

    def _spinor_rhs(self, psi: torch.Tensor) -> int:
        """Validate a canonical spinor tensor; returns its number of right-hand sides."""
        if psi.dtype != torch.complex128 or not psi.is_cuda:
            raise ValueError("spinor must be a complex128 device tensor")
        shape = tuple(psi.shape)
        if shape == self.site_shape + (4, 3):
            return 1
        if len(shape) == 7 and shape[1:] == self.site_shape + (4, 3) and 1 <= shape[0] <= MAX_RHS:
            return shape[0]
        raise ValueError(f"spinor shape {shape} does not match (nrhs,)+{self.site_shape}+(4,3)")

    def _packed_ok(self, t: torch.Tensor, prec, nrhs, parity):
        need = cola_field_bytes(self.h, prec, nrhs, parity)
        if need == 0 or t.dtype != torch.uint8 or not t.is_cuda or t.numel() < need:
            raise ValueError(f"packed buffer must be a device uint8 tensor of >= {need} bytes")

    def pack(self, psi: torch.Tensor, prec, parity=-1) -> torch.Tensor:
        nrhs = self._spinor_rhs(psi)
        out = self.empty_packed(prec, nrhs, parity)
        cola_pack_spinor(self.h, _ptr(out), _ptr(psi.contiguous()), prec, nrhs, parity, _stream())
        return out

    def unpack(self, packed: torch.Tensor, prec, nrhs=1, parity=-1, out=None) -> torch.Tensor:
        self._packed_ok(packed, prec, nrhs, parity)
        if out is None:
            out = torch.zeros((nrhs,) + self.site_shape + (4, 3), dtype=torch.complex128,
                              device="cuda")
        if self._spinor_rhs(out) != nrhs:
            raise ValueError("out has the wrong number of right-hand sides")
        cola_unpack_spinor(self.h, _ptr(out), _ptr(packed), prec, nrhs, parity, _stream())
        return out

    def dslash(self, out: torch.Tensor, inp: torch.Tensor, op, parity=-1, prec=COLA_FP64, nrhs=1):
        full = op in (COLA_OP_M, COLA_OP_MDAG, COLA_OP_MDAGM)
        if nrhs < 1 or nrhs > MAX_RHS or prec not in (0, 1, 2, 3):
            # let the library report the error without touching the buffers
            cola_dslash_apply(self.h, _ptr(out), _ptr(inp), op, parity, prec, nrhs, _stream())
        self._packed_ok(out, prec, nrhs, -1 if full else 0)
        self._packed_ok(inp, prec, nrhs, -1 if full else 0)
        cola_dslash_apply(self.h, _ptr(out), _ptr(inp), op, parity, prec, nrhs, _stream())
        return out

    def cg(self, b: torch.Tensor, system=COLA_SYS_MDAGM, scheme=COLA_CG_FP64, tol=1e-10,
           max_iter=20000, reliable_interval=50, inner_tol=0.0, x0=None, check_interval=0,
           block=0):
        nrhs = self._spinor_rhs(b)
        if x0 is not None and tuple(x0.shape) != tuple(b.shape):
            raise ValueError("x0 must have the shape of b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        p = CgParams(system, scheme, block, tol, max_iter, reliable_interval, inner_tol,
                     0 if x0 is None else 1, check_interval)
        res = (ctypes.c_double * nrhs)()
        r = CgResult(0, 0, 0, 0, ctypes.cast(res, ctypes.POINTER(ctypes.c_double)), 0.0)
        cola_cg_solve(self.h, _ptr(x), _ptr(b.contiguous()), nrhs, p, r, _stream())
        info = {"status": r.status, "iterations": r.iterations, "outer_cycles": r.outer_cycles,
                "reliable_updates": r.reliable_updates, "true_rel_residual": list(res),
                "seconds": r.seconds}
        return x, info

    def _nvec(self, X: torch.Tensor) -> int:
        """Validate a stack of canonical spinors (1 .. 32 of them)."""
        if X.dtype != torch.complex128 or not X.is_cuda:
            raise ValueError("vectors must be a complex128 device tensor")
        shape = tuple(X.shape)
        if len(shape) == 7 and shape[1:] == self.site_shape + (4, 3) and 1 <= shape[0] <= 32:
            return shape[0]
        raise ValueError(f"vector stack shape {shape} is not (n,)+{self.site_shape}+(4,3)")

    def eigensolve(self, X0: torch.Tensor, system=COLA_SYS_SCHUR, tol=1e-8,
                   inner_reduction=0.1, inner_max=50, max_sweeps=100):
        """The len(X0) lowest eigenpairs of A (M^H M or S^H S) from the starting vectors
        X0 (canonical, leading vector axis); returns (eigenvalues, X, info)."""
        n = self._nvec(X0)
        X = X0.contiguous().clone()
        p = EigParams(system, tol, inner_reduction, inner_max, max_sweeps)
        lam = (ctypes.c_double * n)()
        res = (ctypes.c_double * n)()
        r = EigResult(0, 0, 0, ctypes.cast(lam, ctypes.POINTER(ctypes.c_double)),
                      ctypes.cast(res, ctypes.POINTER(ctypes.c_double)), 0.0)
        cola_eigensolve(self.h, _ptr(X), n, p, r, _stream())
        return list(lam), X, {"status": r.status, "sweeps": r.sweeps,
                              "applications": r.applications, "residuals": list(res),
                              "seconds": r.seconds}

    def cg_deflated(self, b: torch.Tensor, X: torch.Tensor, lam, system=COLA_SYS_SCHUR,
                    scheme=COLA_CG_FP64, tol=1e-10, max_iter=20000, reliable_interval=50,
                    inner_tol=0.0, check_interval=0, block=0):
        """cg() started from the low-mode part of the solution (eigenpairs X, lam of the
        same system's A)."""
        nrhs = self._spinor_rhs(b)
        n = self._nvec(X)
        x = torch.zeros_like(b)
        p = CgParams(system, scheme, block, tol, max_iter, reliable_interval, inner_tol, 1,
                     check_interval)
        res = (ctypes.c_double * nrhs)()
        r = CgResult(0, 0, 0, 0, ctypes.cast(res, ctypes.POINTER(ctypes.c_double)), 0.0)
        Xc = X.contiguous()
        cola_cg_deflated(self.h, _ptr(x), _ptr(b.contiguous()), nrhs, _ptr(Xc), list(lam), n, p,
                         r, _stream())
        return x, {"status": r.status, "iterations": r.iterations,
                   "outer_cycles": r.outer_cycles, "true_rel_residual": list(res),
                   "seconds": r.seconds}

    def cg_multishift(self, b: torch.Tensor, shifts, system=COLA_SYS_MDAGM, tol=1e-10,
                      max_iter=20000):
        """(A + shifts[q]) x_q = b for every shift from one Krylov space (FP64); returns
        x with a leading shift axis and the solver info."""
        if self._spinor_rhs(b) != 1:
            raise ValueError("multi-shift CG takes one right-hand side")
        n = len(shifts)
        x = torch.zeros((n,) + self.site_shape + (4, 3), dtype=torch.complex128, device="cuda")
        p = CgParams(system, COLA_CG_FP64, 0, tol, max_iter, 50, 0.0, 0, 0)
        res = (ctypes.c_double * n)()
        r = CgResult(0, 0, 0, 0, ctypes.cast(res, ctypes.POINTER(ctypes.c_double)), 0.0)
        bc = b.reshape(self.site_shape + (4, 3)).contiguous()  # alive through the call
        cola_cg_multishift(self.h, _ptr(x), _ptr(bc), n, shifts, p, r, _stream())
        return x, {"status": r.status, "iterations": r.iterations,
                   "true_rel_residual": list(res), "seconds": r.seconds}

    def force(self, X: torch.Tensor, Y: torch.Tensor, mode=COLA_FORCE_GRAD) -> torch.Tensor:
        if self._spinor_rhs(X) != 1 or self._spinor_rhs(Y) != 1:
            raise ValueError("force takes single-rhs X and Y")
        F = torch.empty(self.site_shape + (4, 3, 3), dtype=torch.complex128, device="cuda")
        cola_fermion_force(self.h, _ptr(F), _ptr(X.contiguous()), _ptr(Y.contiguous()), mode,
                           _stream())
        return F

    # ------------------------------------------------------------------ HMC
    def _gauge_like(self, A: torch.Tensor, name: str):
        if A.dtype != torch.complex128 or tuple(A.shape) != self.site_shape + (4, 3, 3) \
                or not A.is_contiguous() or not A.is_cuda:
            raise ValueError(f"{name} must be contiguous complex128 (Lt,Lz,Ly,Lx,4,3,3) on the GPU")

    def ape_smear(self, U: torch.Tensor, alpha: float, nsweeps: int) -> torch.Tensor:
        """APE-smeared copy of U (nsweeps sweeps of weight alpha, SU(3)-projected)."""
        self._gauge_like(U, "U")
        F = torch.empty_like(U)
        cola_ape_smear(self.h, _ptr(F), _ptr(U.contiguous()), float(alpha), int(nsweeps),
                       _stream())
        return F

    def set_fat_gauge(self, F: torch.Tensor):
        """Switch to the FLIC operator with smeared links F (thin links from set_gauge)."""
        self._gauge_like(F, "F")
        cola_set_fat_gauge(self.h, _ptr(F.contiguous()), _stream())

    def gauge_force(self, U: torch.Tensor, beta: float) -> torch.Tensor:
        self._gauge_like(U, "U")
        F = torch.empty_like(U)
        cola_gauge_force(self.h, _ptr(F), _ptr(U), beta, _stream())
        return F

    def gauge_action(self, U: torch.Tensor, beta: float) -> float:
        self._gauge_like(U, "U")
        return cola_gauge_action(self.h, _ptr(U), beta, _stream())

    def link_update(self, U: torch.Tensor, P: torch.Tensor, eps: float):
        """U <- exp(i eps P) U in place."""
        self._gauge_like(U, "U")
        self._gauge_like(P, "P")
        cola_link_update(self.h, _ptr(U), _ptr(P), eps, _stream())

    def momentum_update(self, P: torch.Tensor, F1: torch.Tensor, eps: float, F2=None):
        """P -= eps (F1 + F2) in place."""
        for A, n in ((P, "P"), (F1, "F1")) + (((F2, "F2"),) if F2 is not None else ()):
            self._gauge_like(A, n)
        cola_momentum_update(self.h, _ptr(P), _ptr(F1), _ptr(F2) if F2 is not None else None,
                             eps, _stream())

    def hmc_trajectory(self, U: torch.Tensor, P: torch.Tensor, beta: float, eps: float,
                       nsteps: int, phi=None, cg_tol=1e-12, cg_max_iter=20000, eo=False,
                       integrator="leapfrog", cg_scheme=COLA_CG_FP64, n_gauge=1) -> dict:
        """One trajectory in place on U and P (phi: pseudofermion or None; eo: the even-odd
        pseudofermion action; integrator: "leapfrog", "omelyan" or "leapfrog_mts" with
        n_gauge gauge sub-steps per fermion step)."""
        kinds = {"leapfrog": 0, "omelyan": 1, "leapfrog_mts": 2}
        if integrator not in kinds:
            raise ValueError(f"integrator must be one of {sorted(kinds)}")
        self._gauge_like(U, "U")
        self._gauge_like(P, "P")
        if phi is not None:
            if self._spinor_rhs(phi) != 1:
                raise ValueError("phi must be one canonical spinor")
            phi = phi.contiguous()
        prm = HmcParams(float(beta), float(eps), int(nsteps), float(cg_tol), int(cg_max_iter),
                        1 if eo else 0, kinds[integrator], int(n_gauge), int(cg_scheme))
        r = HmcResult()
        cola_hmc_trajectory(self.h, _ptr(U), _ptr(P), _ptr(phi) if phi is not None else None,
                            prm, r, _stream())
        return {k: getattr(r, k) for k, _ in HmcResult._fields_}

    def stats(self, prec=None) -> dict:
        """Hop accounting for one precision, or summed over all when prec is None; "kinds"
        splits it by launch kind (COLA_HOP_*: launches, seconds, algorithmic bytes)."""
        s = cola_get_stats(self.h)
        idx = range(4) if prec is None else [prec]
        kinds = {}
        for k in range(HOP_KINDS):
            n = sum(s.kind_launches[i][k] for i in idx)
            if n:
                kinds[k] = {"launches": n, "seconds": sum(s.kind_seconds[i][k] for i in idx),
                            "bytes": sum(s.kind_bytes[i][k] for i in idx)}
        return {"hop_launches": sum(s.hop_launches[i] for i in idx),
                "hop_seconds": sum(s.hop_seconds[i] for i in idx),
                "hop_bytes": sum(s.hop_bytes[i] for i in idx),
                "hop_flops": sum(s.hop_flops[i] for i in idx),
                "kinds": kinds}

    def reset_stats(self):
        cola_reset_stats(self.h)


class PseudofermionAction(torch.autograd.Function):
    """S(U) = phi^H (M^H M)^{-1} phi for plain Wilson M; backward gives dS/dU.

    forward: one cola_fermion_action call (X = (M^H M)^{-1} phi by FP64 CG, Y = M X,
    S = Re <phi, X>, all on the device).
    backward: grad_U = gS * (dS/dRe U + i dS/dIm U) from the link-wise adjoint
    kernel; phi receives no gradient.
    """

    @staticmethod
    def forward(ctx, U, phi, lattice: Lattice, tol=1e-12):
        lattice.set_gauge(U.detach())
        phi_c = phi.detach().contiguous()
        if lattice._spinor_rhs(phi_c) != 1:
            raise ValueError("phi must be one canonical spinor")
        X = torch.empty_like(phi_c)
        Y = torch.empty_like(phi_c)
        rc, S, iters = cola_fermion_action(lattice.h, _ptr(phi_c), _ptr(X), _ptr(Y), tol,
                                           _stream())
        if rc != COLA_OK:
            raise ColaError(rc, f"CG did not converge in {iters} iterations")
        ctx.lattice = lattice
        ctx.save_for_backward(X, Y)
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gS):
        X, Y = ctx.saved_tensors
        G = ctx.lattice.force(X, Y, COLA_FORCE_GRAD)
        return gS * G, None, None, None
