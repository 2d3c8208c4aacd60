"""FP64 CPU oracle for multi-shift CG (plain numpy; TEST INFRASTRUCTURE ONLY).

Solves (A + sigma_i) x_i = b for several shifts sigma_i >= 0 at once, A = M^H M on
the full lattice (system 0) or S^H S on the even sites (system 1), from one Krylov
space (the shifted solver behind rational HMC, which the paper lists with Kennedy et
al.).  The shifted residuals stay collinear with the unshifted CG residual,
r_i = zeta_i r, and the zeta recursion follows from the CG recurrences: with the base
CG's alpha_k, beta_k (r_k+1 = r_k - alpha_k A p_k, p_k+1 = r_k+1 + beta_k p_k),

  zeta_i' = zeta_i zeta_i^old alpha^old /
            (alpha beta^old (zeta_i^old - zeta_i) + zeta_i^old alpha^old (1 + sigma_i alpha))
  alpha_i = alpha zeta_i' / zeta_i,   x_i += alpha_i p_i
  beta_i  = beta (zeta_i' / zeta_i)^2, p_i = zeta_i' r' + beta_i p_i

starting from zeta = zeta^old = 1, alpha^old = 1, beta^old = 0, p_i = b.  The base
system is the unshifted A; the iteration stops when every shifted residual
|zeta_i| |r| is at most tol |b| (|zeta_i| <= 1 for sigma_i >= 0).
"""
from __future__ import annotations

import numpy as np

import oracle


def apply_A(U, v, kappa, bc, system, clover=None, clover_inv=None):
    if system == 0:
        return oracle.apply_M(U, oracle.apply_M(U, v, kappa, bc, clover=clover), kappa, bc,
                              clover=clover, dagger=True)
    t = oracle.apply_schur(U, v, kappa, bc, clover, clover_inv)
    return oracle.apply_schur(U, t, kappa, bc, clover, clover_inv, dagger=True)


def multishift_cg(U, b, shifts, kappa, bc, system=0, tol=1e-10, max_iter=10000, clover=None,
                  clover_inv=None):
    """Returns (x[nshift], iterations).  For system 1 only the even sites of b are used."""
    shifts = np.asarray(shifts, dtype=np.float64)
    if np.any(shifts < 0):
        raise ValueError("shifts must be >= 0")
    if system == 1:
        b = np.where(oracle.parity_mask(b.shape[:4][::-1])[..., None, None], b, 0)
    n = len(shifts)
    x = np.zeros((n,) + b.shape, dtype=np.complex128)
    r = b.copy()
    p = b.copy()
    ps = np.repeat(b[None], n, axis=0)
    zeta = np.ones(n)
    zeta_old = np.ones(n)
    alpha_old, beta_old = 1.0, 0.0
    rho = float(np.real(np.vdot(r, r)))
    bnorm2 = rho
    done = np.zeros(n, dtype=bool)
    it = 0
    while it < max_iter and not np.all(done):
        Ap = apply_A(U, p, kappa, bc, system, clover, clover_inv)
        alpha = rho / float(np.real(np.vdot(p, Ap)))
        zeta_new = zeta * zeta_old * alpha_old / (
            alpha * beta_old * (zeta_old - zeta) + zeta_old * alpha_old * (1 + shifts * alpha))
        alpha_s = alpha * zeta_new / zeta
        for i in range(n):
            if not done[i]:
                x[i] += alpha_s[i] * ps[i]
        r = r - alpha * Ap
        rho_new = float(np.real(np.vdot(r, r)))
        beta = rho_new / rho
        beta_s = beta * (zeta_new / zeta) ** 2
        for i in range(n):
            if not done[i]:
                ps[i] = zeta_new[i] * r + beta_s[i] * ps[i]
        p = r + beta * p
        zeta_old, zeta = zeta, zeta_new
        alpha_old, beta_old, rho = alpha, beta, rho_new
        it += 1
        done |= zeta ** 2 * rho <= tol * tol * bnorm2
    return x, it
