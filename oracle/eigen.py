"""FP64 CPU oracle for the low-eigenmode solver and deflated CG (plain numpy).

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone; it shares no code with
the GPU library.

The paper lists solvers for eigenmodes beside the linear-system solvers among COLA's
key algorithms, citing Kalkreuter and Simma's accelerated conjugate-gradient method
for low-lying eigenvalues of lattice Dirac operators.  That method, restated here in
this module's notation, finds the n smallest eigenpairs (lambda_i, x_i) of a Hermitian
positive operator A -- here A = M^H M on the full lattice (system 0) or S^H S on the
even sites (system 1) -- by minimising Rayleigh quotients:

  sweep: for i = 0 .. n-1
      x <- x_i with the components along x_0 .. x_{i-1} removed, normalised;
      minimise mu(x) = <x, A x> over unit vectors orthogonal to x_0 .. x_{i-1} by
      conjugate gradients: the gradient direction g = P (A x - mu x) (P the projector
      onto the complement of x_0 .. x_{i-1}), the search direction p = g + beta p
      (beta = |g|^2 / |g_old|^2), and an exact line search on the unit circle spanned
      by x and the part q of p orthogonal to x (the lower eigenvector of the 2 x 2
      matrix of A on {x, q}), one application of A per iteration;
      the minimisation of each vector stops early -- the acceleration -- once |g| has
      fallen by the factor `inner_reduction` (or after `inner_max` iterations);
  then diagonalise A on the span of the n vectors (Rayleigh-Ritz: H = X^H A X,
  H = W diag(lambda) W^H, X <- X W, eigenvalues ascending), and repeat sweeps until
  every |A x_i - lambda_i x_i| <= tol * lambda_i.

Deflated CG (the use of the low modes in a solve): the initial guess is the low-mode
part of the solution, x_0 = sum_i x_i <x_i, b> / lambda_i, and plain CG continues from
there; with exact eigenpairs the residual b - A x_0 has no component along them.
"""
from __future__ import annotations

import numpy as np

import oracle

from .multishift import apply_A


def _even(v, system):
    if system != 1:
        return v
    return np.where(oracle.parity_mask(v.shape[:4][::-1])[..., None, None], v, 0)


def _dot(a, b):
    return np.vdot(a, b)


def eigensolve(U, X0, kappa, bc, system=1, tol=1e-8, inner_reduction=0.1, inner_max=50,
               max_sweeps=100, clover=None, clover_inv=None):
    """Lowest n = len(X0) eigenpairs of A from the starting vectors X0 (canonical spinors,
    shape (n, Lt, Lz, Ly, Lx, 4, 3); system 1 uses their even sites only).

    Returns (lambda[n] ascending, X[n] orthonormal, sweeps, operator applications)."""
    X = np.array([_even(np.asarray(x, dtype=np.complex128), system) for x in X0])
    n = len(X)

    def A(v):
        return _even(apply_A(U, v, kappa, bc, system, clover, clover_inv), system)

    napply = 0
    lam = np.zeros(n)
    Y = np.zeros_like(X)
    for sweep in range(1, max_sweeps + 1):
        for i in range(n):
            x = X[i].copy()
            for j in range(i):
                x -= X[j] * _dot(X[j], x)
            x /= np.linalg.norm(x)

            def proj(v):
                for j in range(i):
                    v = v - X[j] * _dot(X[j], v)
                return v

            y = A(x)
            napply += 1
            mu = float(np.real(_dot(x, y)))
            g = proj(y - mu * x)
            gn2 = float(np.real(_dot(g, g)))
            g0 = np.sqrt(gn2)
            p = g.copy()
            for _ in range(inner_max):
                if not gn2 > 0.0:
                    break
                q = proj(p)
                q = q - x * _dot(x, q)
                qn = np.linalg.norm(q)
                if not qn > 0.0:
                    break
                q /= qn
                z = A(q)
                napply += 1
                b = _dot(x, z)
                c = float(np.real(_dot(q, z)))
                w, V = np.linalg.eigh(np.array([[mu, b], [np.conj(b), c]]))
                u0, u1 = V[0, 0], V[1, 0]
                x = u0 * x + u1 * q
                y = u0 * y + u1 * z
                nx = np.linalg.norm(x)
                x /= nx
                y /= nx
                mu = float(np.real(_dot(x, y)))
                gnew = proj(y - mu * x)
                gnew2 = float(np.real(_dot(gnew, gnew)))
                if np.sqrt(gnew2) <= inner_reduction * g0:
                    gn2 = gnew2
                    break
                p = gnew + (gnew2 / gn2) * p
                gn2 = gnew2
            X[i] = x
            Y[i] = y
        # Rayleigh-Ritz on the span of the sweep's vectors
        H = np.array([[_dot(X[a], Y[b]) for b in range(n)] for a in range(n)])
        H = 0.5 * (H + H.conj().T)
        lam, W = np.linalg.eigh(H)
        X = np.tensordot(W.T, X, axes=1)
        Y = np.tensordot(W.T, Y, axes=1)
        res = np.array([np.linalg.norm(Y[i] - lam[i] * X[i]) for i in range(n)])
        if np.all(res <= tol * np.abs(lam)):
            return lam, X, sweep, napply
    return lam, X, max_sweeps, napply


def deflated_guess(X, lam, b, system=1):
    """x_0 = sum_i x_i <x_i, b> / lambda_i (b's even sites for system 1)."""
    b = _even(np.asarray(b, dtype=np.complex128), system)
    x0 = np.zeros_like(b)
    for xi, li in zip(X, lam):
        x0 += xi * (_dot(xi, b) / li)
    return x0


def cg_from(U, b, x0, kappa, bc, system=1, tol=1e-10, max_iter=10000, clover=None,
            clover_inv=None):
    """Plain CG on A x = b from x0; stops when the true relative residual |b - A x|/|b|
    is at most tol.  Returns (x, iterations)."""
    b = _even(np.asarray(b, dtype=np.complex128), system)

    def A(v):
        return _even(apply_A(U, v, kappa, bc, system, clover, clover_inv), system)

    x = np.array(x0, dtype=np.complex128)
    r = b - A(x)
    p = r.copy()
    rho = float(np.real(_dot(r, r)))
    bn2 = float(np.real(_dot(b, b)))
    it = 0
    while it < max_iter:
        if rho <= tol * tol * bn2:
            rt = b - A(x)
            if float(np.real(_dot(rt, rt))) <= tol * tol * bn2:
                break
            r = rt
            rho = float(np.real(_dot(r, r)))
            p = r.copy()
        Ap = A(p)
        alpha = rho / float(np.real(_dot(p, Ap)))
        x = x + alpha * p
        r = r - alpha * Ap
        rho_new = float(np.real(_dot(r, r)))
        p = r + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it
