"""Pins of the low-eigenmode oracle (accelerated CG on Rayleigh quotients) and of
deflated CG.

Against dense eigendecompositions of A = M^H M and S^H S on a 2x2x2x4 lattice (an
extent-2 direction included), the free-field spectrum of S^H S in closed form, gauge
invariance of the spectrum, and for deflated CG dense solves and the iteration count
of plain CG from zero.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, eigen
from paper_2302_00850_amd.synth import Synth, bc_phases, unit_gauge
from tests._util import rel

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
ANTI = bc_phases((0, 0, 0, np.pi))


def _dense_A(U, kappa, bc, dims, system):
    M = dense.wilson_matrix(U, kappa, bc)
    if system == 0:
        return M.conj().T @ M, np.ones(M.shape[0], dtype=bool)
    S = dense.schur_matrix(M, dims)
    return S.conj().T @ S, dense.parity_vector(dims) == 0


@pytest.mark.parametrize("system", [0, 1])
def test_eigenpairs_match_dense_eigh(system):
    dims = (2, 2, 2, 4)
    s = Synth(61)
    U = s.gauge(dims, mix=0.6).numpy()
    n = 6
    X0 = s.gaussian_spinor(dims, n).numpy()
    kappa = 0.11
    lam, X, sweeps, napply = eigen.eigensolve(U, X0, kappa, GENERIC, system=system, tol=1e-9)
    A, rows = _dense_A(U, kappa, GENERIC, dims, system)
    w, V = np.linalg.eigh(A)
    assert np.all(np.abs(lam - w[:n]) <= 1e-10 * w[:n]), (lam, w[:n])
    Xv = np.array([dense.to_vec(x)[rows] for x in X])
    # orthonormal, and each a true eigenvector to the tolerance
    assert np.abs(Xv.conj() @ Xv.T - np.eye(n)).max() < 1e-12
    for i in range(n):
        assert np.linalg.norm(A @ Xv[i] - lam[i] * Xv[i]) <= 1e-9 * lam[i]
    # the same invariant subspace as the dense one (a gap follows the n-th eigenvalue)
    assert w[n] - w[n - 1] > 1e-3 * w[n]
    P_got = Xv.T @ Xv.conj()
    P_ref = V[:, :n] @ V[:, :n].conj().T
    assert np.abs(P_got - P_ref).max() < 1e-8
    if system == 1:
        assert all(np.all(dense.to_vec(x)[~rows] == 0) for x in X)


def _free_schur_spectrum(dims, kappa, theta):
    """Eigenvalues of S^H S at U = 1 with multiplicity: per momentum p (p_mu = (2 pi n_mu +
    theta_mu) / L_mu) the hop symbol is c - i g.s with c = sum 2 cos p_mu, s_mu = 2 sin p_mu;
    D^2 has the eigenvalues (c -+ i|s|)^2, so S = 1 - kappa^2 D^2 on the even sites gives
    |1 - kappa^2 (c -+ i|s|)^2|^2 (equal for both signs), 6 times per p over all V momenta."""
    ps = [(2 * np.pi * np.arange(L) + th) / L for L, th in zip(dims, theta)]
    px, py, pz, pt = np.meshgrid(*ps, indexing="ij")
    c = 2 * (np.cos(px) + np.cos(py) + np.cos(pz) + np.cos(pt))
    s = 2 * np.sqrt(np.sin(px) ** 2 + np.sin(py) ** 2 + np.sin(pz) ** 2 + np.sin(pt) ** 2)
    lam = np.abs(1 - kappa ** 2 * (c - 1j * s) ** 2) ** 2
    return np.sort(np.repeat(lam.ravel(), 6))


def test_free_field_spectrum():
    dims = (2, 2, 2, 4)
    kappa = 0.12
    theta = (0.3, -0.5, 0.7, np.pi)
    U = unit_gauge(dims).numpy()
    # the lowest free-field level is 24-fold here: 28 vectors reach into the next one
    n = 28
    X0 = Synth(62).gaussian_spinor(dims, n).numpy()
    lam, X, _, _ = eigen.eigensolve(U, X0, kappa, GENERIC, system=1, tol=1e-9)
    ref = _free_schur_spectrum(dims, kappa, theta)
    assert len(ref) == 6 * int(np.prod(dims))
    assert np.abs(lam - ref[:n]).max() <= 1e-10 * ref[n - 1]
    assert ref[n - 1] > ref[0] * 1.5
    # and the closed form agrees with the dense matrix on this lattice
    A, _ = _dense_A(U, kappa, GENERIC, dims, 1)
    assert np.abs(np.linalg.eigvalsh(A) - ref).max() < 1e-12


def test_spectrum_gauge_invariant():
    dims = (4, 4, 2, 4)
    s = Synth(63)
    U = s.gauge(dims).numpy()
    G = s.haar_field(dims).numpy()
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    n = 4
    X0 = s.gaussian_spinor(dims, n).numpy()
    lam, _, _, _ = eigen.eigensolve(U, X0, 0.12, GENERIC, system=1, tol=1e-9)
    X0G = np.einsum("tzyxab,ntzyxsb->ntzyxsa", G, X0)
    lamG, _, _, _ = eigen.eigensolve(UG, X0G, 0.12, GENERIC, system=1, tol=1e-9)
    assert np.abs(lam - lamG).max() <= 1e-9 * lam.max()


@pytest.mark.parametrize("system", [0, 1])
def test_deflated_cg(system):
    dims = (2, 2, 2, 4)
    s = Synth(64)
    U = s.gauge(dims, mix=0.6).numpy()
    kappa = 0.124
    n = 8
    X0 = s.gaussian_spinor(dims, n).numpy()
    b = s.gaussian_spinor(dims).numpy()[0]
    lam, X, _, _ = eigen.eigensolve(U, X0, kappa, GENERIC, system=system, tol=1e-11)
    x0 = eigen.deflated_guess(X, lam, b, system)
    A, rows = _dense_A(U, kappa, GENERIC, dims, system)
    bv = dense.to_vec(b)[rows]
    r0 = bv - A @ dense.to_vec(x0)[rows]
    # the starting residual has no component along the low modes
    Xv = np.array([dense.to_vec(x)[rows] for x in X])
    assert np.abs(Xv.conj() @ r0).max() <= 1e-9 * np.linalg.norm(bv)
    x, it = eigen.cg_from(U, b, x0, kappa, GENERIC, system, tol=1e-12)
    assert rel(dense.to_vec(x)[rows], np.linalg.solve(A, bv)) < 1e-9
    _, it0 = eigen.cg_from(U, b, np.zeros_like(b), kappa, GENERIC, system, tol=1e-12)
    assert it < it0, (it, it0)
