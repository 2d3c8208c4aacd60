"""Dense brute-force Wilson-Dirac matrices on tiny lattices (numpy).

TEST INFRASTRUCTURE ONLY.  A third, independent route to the operator: the
whole matrix M (12V x 12V) is assembled block by block from the textbook
definition

  M = 1 - kappa sum_x sum_mu [ |x><x+mu| (x) (1 - g_mu) (x) e+ U_mu(x)
                              + |x><x-mu| (x) (1 + g_mu) (x) e- U_mu(x-mu)^H ]

(row/column index = 12*site + 3*spin + colour, site = x + Lx(y + Lz(..)),
boundary phase e+ = exp(i theta_mu) on the hop out of x_mu = L_mu - 1, e- its
conjugate on the hop out of x_mu = 0).  On an extent-2 direction the forward
and backward neighbours are the same site and both blocks are added.

Everything else here -- solves, Schur complements, the action S used for
finite differences -- is plain dense linear algebra on that matrix.
"""
from __future__ import annotations

import numpy as np

# chiral (DeGrand-Rossi) basis, mu = 0..3 = x, y, z, t
_G = [
    np.array([[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]]),
    np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=complex),
    np.array([[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]]),
    np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=complex),
]


def gammas():
    return [g.copy() for g in _G]


def gamma5():
    return _G[0] @ _G[1] @ _G[2] @ _G[3]


def _sites(dims):
    lx, ly, lz, lt = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    yield (x, y, z, t)


def _index(dims, c):
    lx, ly, lz, _ = dims
    return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))


def dims_of(U):
    lt, lz, ly, lx = U.shape[:4]
    return (lx, ly, lz, lt)


def _link(U, c, mu):
    return U[c[3], c[2], c[1], c[0], mu]


def hop_matrix(U, bc):
    """The dense hopping matrix D (so that M = 1 - kappa D)."""
    U = np.asarray(U)
    dims = dims_of(U)
    V = int(np.prod(dims))
    phase = np.asarray(bc, dtype=float).reshape(4, 2)
    phase = phase[:, 0] + 1j * phase[:, 1]
    D = np.zeros((12 * V, 12 * V), dtype=complex)
    one = np.eye(4)
    for c in _sites(dims):
        i = _index(dims, c)
        for mu in range(4):
            fwd = list(c)
            fwd[mu] = (c[mu] + 1) % dims[mu]
            bwd = list(c)
            bwd[mu] = (c[mu] - 1) % dims[mu]
            ef = phase[mu] if c[mu] == dims[mu] - 1 else 1.0
            eb = np.conj(phase[mu]) if c[mu] == 0 else 1.0
            jf, jb = _index(dims, fwd), _index(dims, bwd)
            D[12 * i:12 * i + 12, 12 * jf:12 * jf + 12] += np.kron(one - _G[mu], ef * _link(U, c, mu))
            D[12 * i:12 * i + 12, 12 * jb:12 * jb + 12] += np.kron(
                one + _G[mu], eb * _link(U, bwd, mu).conj().T)
    return D


def wilson_matrix(U, kappa, bc, clover=None):
    """Dense M = A - kappa D; clover is an optional (Lt,Lz,Ly,Lx,12,12) site-matrix field."""
    D = hop_matrix(U, bc)
    n = D.shape[0]
    if clover is None:
        A = np.eye(n, dtype=complex)
    else:
        A = np.zeros((n, n), dtype=complex)
        dims = dims_of(U)
        for c in _sites(dims):
            i = _index(dims, c)
            A[12 * i:12 * i + 12, 12 * i:12 * i + 12] = clover[c[3], c[2], c[1], c[0]]
    return A - kappa * D


def parity_vector(dims):
    """Per-row parity (0 even, 1 odd) in the dense index order."""
    par = np.empty(12 * int(np.prod(dims)), dtype=int)
    for c in _sites(dims):
        i = _index(dims, c)
        par[12 * i:12 * i + 12] = sum(c) % 2
    return par


def schur_matrix(M, dims):
    """S = M_ee - M_eo M_oo^{-1} M_oe, with the even rows/cols in dense order."""
    par = parity_vector(dims)
    e, o = par == 0, par == 1
    Mee, Meo, Moe, Moo = M[np.ix_(e, e)], M[np.ix_(e, o)], M[np.ix_(o, e)], M[np.ix_(o, o)]
    return Mee - Meo @ np.linalg.solve(Moo, Moe)


def to_vec(psi):
    """Canonical spinor (Lt,Lz,Ly,Lx,4,3) -> dense vector."""
    return np.asarray(psi).reshape(-1)


def from_vec(v, dims):
    lx, ly, lz, lt = dims
    return np.asarray(v).reshape(lt, lz, ly, lx, 4, 3)


def action(U, phi, kappa, bc):
    """S = phi^H (M^H M)^{-1} phi, by a dense solve."""
    M = wilson_matrix(U, kappa, bc)
    v = to_vec(phi)
    y = np.linalg.solve(M.conj().T, v)  # (M^H)^{-1} phi
    return float(np.vdot(y, y).real)
