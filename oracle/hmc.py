"""FP64 CPU oracle for one HMC trajectory (plain numpy; TEST INFRASTRUCTURE ONLY).

Hybrid Monte Carlo (the gauge-field generation method the paper lists among its
algorithms, with the Duane et al. reference) for SU(3) links with the Wilson gauge
action and, optionally, two flavours of plain Wilson fermions through one
pseudofermion field:

  H(U, P) = sum_links Tr(P^2) / 2 + S_g(U) + S_f(U)
  S_g = beta sum_{x, mu<nu} (1 - Re Tr U_mu,nu(x) / 3)       (plaquette action)
  S_f = phi^H (M^H M)^{-1} phi                               (M = 1 - kappa D)
     or phi_e^H (S^H S)^{-1} phi_e on the even sites          (S = 1 - kappa^2 D_eo D_oe)

P is traceless Hermitian per link.  A link moves as U -> exp(i eps P) U and the
force F(U) is the traceless Hermitian matrix with dS/de = Tr(H F) along
U -> exp(i e H) U, so that dP/dtau = -F conserves H.  Integrators: leapfrog (half
step in P, n alternating full steps, half step in P) and the second-order
minimum-norm (Omelyan) scheme, whose coefficient lambda minimises the norm of the
leading error terms.

Nothing here is shared with the GPU library; the fermion parts call the C oracle
(CG, M and the fermion force in its Lie-algebra form).
"""
from __future__ import annotations

import numpy as np

import oracle


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def _shift(a, mu, s):
    """b(x) = a(x + s mu) on the periodic lattice (arrays indexed [t][z][y][x])."""
    return np.roll(a, -s, axis=3 - mu)


def plaquettes(U):
    """U_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H for mu < nu."""
    out = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = U[..., mu, :, :], U[..., nu, :, :]
            out[mu, nu] = Um @ _shift(Un, mu, 1) @ _dag(_shift(Um, nu, 1)) @ _dag(Un)
    return out


def gauge_action(U, beta):
    """Wilson plaquette action beta sum (1 - Re Tr U_plaq / 3)."""
    s = 0.0
    for P in plaquettes(U).values():
        s += np.sum(1.0 - np.real(np.einsum("...ii->...", P)) / 3.0)
    return beta * s


def staples(U, mu):
    """A_mu(x) with sum over plaquettes containing U_mu(x) of Re Tr = Re Tr(U_mu(x) A_mu(x)):
    for each nu != mu the upper staple U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H and the lower
    one U_nu(x+mu-nu)^H U_mu(x-nu)^H U_nu(x-nu)."""
    A = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
    Um = U[..., mu, :, :]
    for nu in range(4):
        if nu == mu:
            continue
        Un = U[..., nu, :, :]
        A += _shift(Un, mu, 1) @ _dag(_shift(Um, nu, 1)) @ _dag(Un)
        Un_m = _shift(Un, nu, -1)                      # U_nu(x - nu)
        A += _dag(_shift(Un_m, mu, 1)) @ _dag(_shift(Um, nu, -1)) @ Un_m
    return A


def traceless_hermitian(X):
    H = 0.5 * (X + _dag(X))
    tr = np.einsum("...ii->...", H)
    return H - tr[..., None, None] / 3.0 * np.eye(3)


def gauge_force(U, beta):
    """F_mu(x) for S_g: with W = U_mu(x) A_mu(x), dS_g/de along exp(i e H) U_mu(x) is
    -(beta/3) Re Tr(i H W) = Tr(H F) for F = -(beta/3) P_TH[i (W - W^H) / 2]."""
    F = np.empty_like(U)
    for mu in range(4):
        W = U[..., mu, :, :] @ staples(U, mu)
        F[..., mu, :, :] = -(beta / 3.0) * traceless_hermitian(0.5j * (W - _dag(W)))
    return F


def expi(P, eps):
    """exp(i eps P) for Hermitian P, from its eigen-decomposition."""
    w, v = np.linalg.eigh(P)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ _dag(v)


def kinetic(P):
    return 0.5 * float(np.sum(np.real(np.einsum("...ij,...ji->...", P, P))))


def _fermion(U, phi, kappa, bc, tol):
    """X = (M^H M)^{-1} phi (FP64 CG), S_f = Re <phi, X> and the Lie-form force."""
    X, _, _ = oracle.cg(U, phi, kappa, bc, system=0, tol=tol)
    Y = oracle.apply_M(U, X, kappa, bc)
    S = float(np.real(np.vdot(phi.ravel(), X.ravel())))
    return S, oracle.force(U, X, Y, kappa, bc, mode=1)


def _fermion_eo(U, phi, kappa, bc, tol):
    """Even-odd pseudofermion S_f = phi_e^H (S^H S)^{-1} phi_e, S = 1 - kappa^2 D_eo D_oe.

    With X_e = (S^H S)^{-1} phi_e and Y_e = S X_e, dS_f = 2 kappa^2 Re[Y_e^H dD_eo X_o +
    Y_o^H dD_oe X_e] for X_o = D_oe X_e and Y_o = (D_eo)^H Y_e: the full-lattice fermion
    force of the vectors (X_e, X_o), (Y_e, Y_o) with kappa^2 in place of kappa."""
    even = oracle.parity_mask(U.shape[:4][::-1])[..., None, None]
    X, _, _ = oracle.cg(U, phi, kappa, bc, system=1, tol=tol)
    X = np.where(even, X, 0)
    S = float(np.real(np.vdot(np.where(even, phi, 0).ravel(), X.ravel())))
    Y = np.where(even, oracle.apply_schur(U, X, kappa, bc), 0)
    Xf = X + np.where(even, 0, oracle.hop(U, X, bc))
    Yf = Y + np.where(even, 0, oracle.hop(U, Y, bc, dagger=True))
    return S, oracle.force(U, Xf, Yf, kappa * kappa, bc, mode=1)


def hamiltonian_and_force(U, P, beta, phi=None, kappa=0.0, bc=None, tol=1e-12, eo=False):
    S = gauge_action(U, beta)
    F = gauge_force(U, beta)
    if phi is not None:
        Sf, Ff = (_fermion_eo if eo else _fermion)(U, phi, kappa, bc, tol)
        S += Sf
        F = F + Ff
    return kinetic(P) + S, F


# second-order minimum-norm (Omelyan) coefficient
OMELYAN_LAMBDA = 0.1931833275037836


def trajectory(U, P, beta, eps, nsteps, phi=None, kappa=0.0, bc=None, tol=1e-12, eo=False,
               integrator="leapfrog", n_gauge=1):
    """One trajectory of nsteps steps of size eps.  Returns (U', P', H0, H1); the inputs
    are not modified.  eo: the even-odd pseudofermion action.  integrator: "leapfrog"
    (P eps/2, U eps, P eps/2 per step), "omelyan" (P lambda eps, U eps/2,
    P (1 - 2 lambda) eps, U eps/2, P lambda eps per step) or "leapfrog_mts" (fermion
    kicks of eps around n_gauge gauge-force leapfrog sub-steps)."""
    U = U.copy()
    P = P.copy()

    def force():
        return hamiltonian_and_force(U, P, beta, phi, kappa, bc, tol, eo)[1]

    def fermion_force():
        if phi is None:
            return np.zeros_like(U)
        return (_fermion_eo if eo else _fermion)(U, phi, kappa, bc, tol)[1]

    def move(h):
        return np.einsum("...ij,...jk->...ik", expi(P, h), U)

    H0, F = hamiltonian_and_force(U, P, beta, phi, kappa, bc, tol, eo)
    if integrator == "leapfrog":
        P -= 0.5 * eps * F
        for k in range(nsteps):
            U = move(eps)
            P -= (eps if k < nsteps - 1 else 0.5 * eps) * force()
    elif integrator == "leapfrog_mts":
        # two time scales (Sexton-Weingarten): the fermion force on steps of eps, the gauge
        # force on n_gauge leapfrog sub-steps of eps / n_gauge between the fermion kicks
        h = eps / n_gauge
        P -= 0.5 * eps * fermion_force()
        for k in range(nsteps):
            P -= 0.5 * h * gauge_force(U, beta)
            for j in range(n_gauge):
                U = move(h)
                P -= (h if j < n_gauge - 1 else 0.5 * h) * gauge_force(U, beta)
            P -= (eps if k < nsteps - 1 else 0.5 * eps) * fermion_force()
    elif integrator == "omelyan":
        lam = OMELYAN_LAMBDA
        P -= lam * eps * F
        for k in range(nsteps):
            U = move(0.5 * eps)
            P -= (1 - 2 * lam) * eps * force()
            U = move(0.5 * eps)
            P -= (lam if k == nsteps - 1 else 2 * lam) * eps * force()
    else:
        raise ValueError("integrator must be 'leapfrog' or 'omelyan'")
    H1, _ = hamiltonian_and_force(U, P, beta, phi, kappa, bc, tol, eo)
    return U, P, H0, H1
