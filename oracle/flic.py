"""FP64 CPU oracle for the fat-link irrelevant clover (FLIC) operator (plain numpy).

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone; it shares no code with the
GPU library.

The paper ties COLA's physics to the CSSM programme, whose fermion action (in the
bibliography's FLIC and fat-link HMC entries) is the fat-link irrelevant clover action:
the relevant, naive part of the Dirac operator uses the gauge links U themselves, and the
irrelevant parts -- the Wilson term and the clover term -- use APE-smeared "fat" links F:

  (M psi)(x) = A_F(x) psi(x)
      - kappa sum_mu [ (F_mu(x) - g_mu U_mu(x)) e+_mu(x) psi(x + mu)
                     + (F_mu(x - mu)^H + g_mu U_mu(x - mu)^H) e-_mu(x) psi(x - mu) ]

with A_F = 1 - kappa c_sw sum_{mu<nu} sigma_mu,nu F_mu,nu[F] the clover matrix of the fat
field, the boundary phases e+- as for the Wilson operator, and M^H = g5 M g5.  With F = U
this is the Wilson-clover operator.

APE smearing, one sweep for all links at once:
  V_mu(x) = (1 - alpha) U_mu(x) + (alpha / 6) sum_{nu != mu} [ U_nu(x) U_mu(x + nu) U_nu(x + mu)^H
                                                         + U_nu(x - nu)^H U_mu(x - nu) U_nu(x - nu + mu) ]
  U'_mu(x) = the SU(3) matrix closest to V: the unitary polar factor W = A B^H of the
             singular value decomposition V = A Sigma B^H, divided by det(W)^(1/3)
             (principal cube root),
repeated n times.  Smearing uses the periodic links (boundary phases live in the
operator only).
"""
from __future__ import annotations

import numpy as np

import oracle

from . import dense


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _shift(a, mu, step):
    """a(x + step * mu) for a field with the site axes (t, z, y, x) first."""
    return np.roll(a, -step, axis=3 - mu)


def project_su3(V):
    """Closest SU(3) matrix: polar factor from the SVD, then the determinant's phase out."""
    A, _, Bh = np.linalg.svd(V)
    W = A @ Bh
    d = np.linalg.det(W)
    return W / np.exp(1j * np.angle(d) / 3.0)[..., None, None]


def ape_smear(U, alpha, nsweeps):
    """nsweeps APE sweeps of the canonical gauge field U (Lt,Lz,Ly,Lx,4,3,3)."""
    U = np.array(U, dtype=np.complex128)
    for _ in range(nsweeps):
        V = np.empty_like(U)
        for mu in range(4):
            Um = U[..., mu, :, :]
            S = np.zeros_like(Um)
            for nu in range(4):
                if nu == mu:
                    continue
                Un = U[..., nu, :, :]
                # upper staple U_nu(x) U_mu(x+nu) U_nu(x+mu)^H
                S += Un @ _shift(Um, nu, 1) @ _dag(_shift(Un, mu, 1))
                # lower staple U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu)
                Unb = _shift(Un, nu, -1)
                S += _dag(Unb) @ _shift(Um, nu, -1) @ _shift(Unb, mu, 1)
            V[..., mu, :, :] = project_su3((1.0 - alpha) * Um + (alpha / 6.0) * S)
        U = V
    return U


def _phases(bc, dims, mu):
    """e+ and e- per site as arrays broadcastable over (Lt,Lz,Ly,Lx)."""
    ph = complex(bc[2 * mu], bc[2 * mu + 1]) if np.ndim(bc) == 1 else complex(*bc[mu])
    L = dims[mu]
    shape = [1, 1, 1, 1]
    shape[3 - mu] = L
    coord = np.arange(L).reshape(shape)
    ep = np.where(coord == L - 1, ph, 1.0 + 0j)
    em = np.where(coord == 0, np.conj(ph), 1.0 + 0j)
    return ep, em


def flic_hop(U, F, psi, bc):
    """sum_mu [(F - g U) e+ psi(x+mu) + (F(x-mu)^H + g U(x-mu)^H) e- psi(x-mu)]."""
    U = np.asarray(U)
    F = np.asarray(F)
    psi = np.asarray(psi, dtype=np.complex128)
    lt, lz, ly, lx = U.shape[:4]
    dims = (lx, ly, lz, lt)
    bcv = np.asarray(bc, dtype=np.float64).reshape(-1)
    g = dense.gammas()
    out = np.zeros_like(psi)
    for mu in range(4):
        ep, em = _phases(bcv, dims, mu)
        Um, Fm = U[..., mu, :, :], F[..., mu, :, :]
        pf = _shift(psi, mu, 1) * ep[..., None, None]
        pb = _shift(psi, mu, -1) * em[..., None, None]
        Ub, Fb = _dag(_shift(Um, mu, -1)), _dag(_shift(Fm, mu, -1))
        # colour: links act on the last index; spin: gamma on the spin index
        Fpf = np.einsum("...ab,...sb->...sa", Fm, pf)
        Upf = np.einsum("...ab,...sb->...sa", Um, pf)
        Fpb = np.einsum("...ab,...sb->...sa", Fb, pb)
        Upb = np.einsum("...ab,...sb->...sa", Ub, pb)
        out += Fpf - np.einsum("st,...tc->...sc", g[mu], Upf)
        out += Fpb + np.einsum("st,...tc->...sc", g[mu], Upb)
    return out


def _g5(psi):
    out = np.array(psi, copy=True)
    out[..., 2:, :] *= -1
    return out


def apply_flic(U, F, psi, kappa, bc, csw=0.0, dagger=False):
    """M psi for the FLIC operator (dagger: M^H psi = g5 M g5 psi); one spinor."""
    psi = np.asarray(psi, dtype=np.complex128)
    if dagger:
        return _g5(apply_flic(U, F, _g5(psi), kappa, bc, csw))
    out = -kappa * flic_hop(U, F, psi, bc)
    if csw:
        A = oracle.clover(F, kappa, csw)
        out += np.einsum("...ij,...j->...i", A, psi.reshape(psi.shape[:4] + (12,))).reshape(
            psi.shape)
    else:
        out += psi
    return out
