"""Pins of the oracle's clover term and fermion force.

Clover: A = 1 at U = 1, Hermitian, block-diagonal in chirality, gauge
covariant, and the closed form of a constant abelian flux.  The overall sign
is fixed by tree-level O(a) improvement: in a constant abelian field the clover
term at c_sw = 1 cancels the Wilson term's shift of the would-be zero modes.

Force: finite differences of the action S = phi^H (M^H M)^{-1} phi computed
by dense solves (a route that never touches the oracle's force code), the
identities Y = eta and S = |eta|^2 for phi = M^H eta, and gauge covariance."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle import dense
from paper_2302_00850_amd.synth import Synth, bc_phases, unit_gauge
from tests._util import rel

ANTIPERIODIC = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))


def test_clover_unit_gauge_is_identity():
    dims = (4, 2, 2, 4)
    A = oracle.clover(unit_gauge(dims).numpy(), 0.118, 1.0)
    assert np.array_equal(A, np.broadcast_to(np.eye(12), A.shape))


def test_clover_hermitian_and_chiral_blocks():
    dims = (4, 4, 2, 2)
    U = Synth(31).gauge(dims).numpy()
    A = oracle.clover(U, 0.118, 1.0)
    assert np.abs(A - A.conj().swapaxes(-1, -2)).max() < 1e-15
    # gamma5 = diag(1,1,-1,-1) in spin: the (upper, lower) chiral blocks do not mix
    assert np.abs(A[..., :6, 6:]).max() < 1e-15
    assert np.abs(A[..., 6:, :6]).max() < 1e-15
    # for these smooth fields each 6x6 block is positive definite
    assert np.linalg.eigvalsh(A[..., :6, :6]).min() > 0
    assert np.linalg.eigvalsh(A[..., 6:, 6:]).min() > 0


def test_clover_gauge_covariance():
    dims = (4, 2, 2, 4)
    s = Synth(32)
    U = s.gauge(dims).numpy()
    G = s.haar_field(dims).numpy()
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    A = oracle.clover(U, 0.118, 1.0)
    AG = oracle.clover(UG, 0.118, 1.0)
    # A(x) -> (1_spin (x) G(x)) A(x) (1_spin (x) G(x))^H
    big = np.einsum("st,...ab->...satb", np.eye(4), G).reshape(G.shape[:4] + (12, 12))
    expect = big @ A @ big.conj().swapaxes(-1, -2)
    assert rel(AG, expect) < 1e-14


def test_clover_constant_abelian_flux():
    """U_x(x) = diag(e^{-i phi y}, e^{i phi y}, 1), other links 1, phi = 2 pi / Ly:
    every x-y plaquette is diag(e^{i phi}, e^{-i phi}, 1), so
    F_xy = sin(phi) diag(1, -1, 0), all other F vanish, and
    A = 1 - kappa c_sw sin(phi) sigma_xy (x) diag(1, -1, 0)."""
    dims = (4, 6, 2, 4)
    lx, ly, lz, lt = dims
    phi = 2 * np.pi / ly
    U = unit_gauge(dims).numpy()
    y = np.arange(ly)
    U[:, :, :, :, 0, 0, 0] = np.exp(-1j * phi * y)[None, None, :, None]
    U[:, :, :, :, 0, 1, 1] = np.exp(1j * phi * y)[None, None, :, None]
    Fxy = oracle.field_strength(U, 0, 1)
    np.testing.assert_allclose(Fxy, np.broadcast_to(np.sin(phi) * np.diag([1, -1, 0]), Fxy.shape),
                               atol=1e-14)
    for mu, nu in [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
        assert np.abs(oracle.field_strength(U, mu, nu)).max() < 1e-14
    kappa, csw = 0.118, 1.0
    g = dense.gammas()
    sig = 0.5j * (g[0] @ g[1] - g[1] @ g[0])
    expect = np.eye(12) - kappa * csw * np.sin(phi) * np.kron(sig, np.diag([1, -1, 0]))
    A = oracle.clover(U, kappa, csw)
    np.testing.assert_allclose(A, np.broadcast_to(expect, A.shape), atol=1e-14)


def _constant_flux_gauge(dims, mu, nu, flux=1):
    """U(1) field of constant strength f = 2 pi flux / (L_mu L_nu) in the (mu, nu) plane,
    embedded as diag(e^{i th}, e^{-i th}, 1): U_nu(x) carries th = f x_mu, and U_mu at
    x_mu = L_mu - 1 carries th = -f L_mu x_nu (the torus twist), every other link is 1.
    Every (mu, nu) plaquette is then e^{i f} on colour 0."""
    L = dims
    f = 2 * np.pi * flux / (L[mu] * L[nu])
    U = unit_gauge(dims).numpy()
    shape = (L[3], L[2], L[1], L[0])
    xm = np.arange(L[mu]).reshape([-1 if 3 - a == mu else 1 for a in range(4)])
    xn = np.arange(L[nu]).reshape([-1 if 3 - a == nu else 1 for a in range(4)])
    th_nu = np.broadcast_to(f * xm, shape)
    th_mu = np.broadcast_to(np.where(xm == L[mu] - 1, -f * L[mu] * xn, 0.0 * xn), shape)
    for d, th in ((nu, th_nu), (mu, th_mu)):
        U[..., d, 0, 0] = np.exp(1j * th)
        U[..., d, 1, 1] = np.exp(-1j * th)
    return U, f


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
def test_clover_cancels_the_wilson_pauli_term(mu, nu):
    """Tree-level O(a) improvement fixes the clover term's overall sign.  In a constant
    abelian field f the massless continuum operator has exact zero modes (index
    theorem; two per unit flux here, for colour 0 constant in the short directions).
    The Wilson term turns them into real eigenvalues f/2 of the massless lattice
    operator 4 - D/2 (its O(a) Pauli term); the clover term at c_sw = 1 exists to
    cancel exactly that, leaving O(f^2); with the opposite sign they move to f."""
    dims = [2, 2, 2, 2]
    dims[mu] = dims[nu] = 8
    dims = tuple(dims)
    U, f = _constant_flux_gauge(dims, mu, nu)
    # the field is what it should be: F_mu_nu = sin(f) diag(1, -1, 0) at every site
    F = oracle.field_strength(U, mu, nu)
    np.testing.assert_allclose(F, np.broadcast_to(np.sin(f) * np.diag([1, -1, 0]), F.shape),
                               atol=1e-13)
    kappa = 0.125
    A = oracle.clover(U, kappa, 1.0)
    V = int(np.prod(dims))
    shape = (dims[3], dims[2], dims[1], dims[0])
    K = np.zeros((4 * V, 4 * V), complex)  # 4 - D/2 on colour 0
    S = np.zeros((4 * V, 4 * V), complex)  # (A - 1) / (2 kappa) on colour 0
    per = bc_phases((0, 0, 0, 0))
    for site in range(V):
        at = np.unravel_index(site, shape)
        for sp in range(4):
            psi = np.zeros(shape + (4, 3), complex)
            psi[at + (sp, 0)] = 1
            K[:, 4 * site + sp] = (4 * psi - 0.5 * oracle.hop(U, psi, per))[..., 0].ravel()
            Ap = np.einsum("...ab,...b->...a", A, psi.reshape(shape + (12,))).reshape(psi.shape)
            S[:, 4 * site + sp] = ((Ap - psi) / (2 * kappa))[..., 0].ravel()

    def lowest(c):
        ev = np.linalg.eigvals(K + c * S)
        return ev[np.argsort(np.abs(ev))[:3]]

    wil, imp, flip = lowest(0.0), lowest(1.0), lowest(-1.0)
    for ev, target in ((wil, f / 2), (flip, f)):
        assert np.abs(ev[:2].imag).max() < 1e-10
        np.testing.assert_allclose(ev[:2].real, target, rtol=0.05)
    assert np.abs(imp[:2]).max() < 0.03 * f / 2
    # the would-be zero modes are isolated from the rest of the spectrum
    for ev in (wil, imp, flip):
        assert np.abs(ev[2]) > 4 * np.abs(ev[1])


# ------------------------------------------------------------------- force

def _solve_xy(U, phi, kappa, bc):
    X, it, res = oracle.cg(U, phi, kappa, bc, system=0, tol=1e-14, max_iter=5000)
    assert it > 0
    return X, oracle.apply_M(U, X, kappa, bc)


@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 4)
    s = Synth(41)
    U = s.gauge(dims).numpy()
    phi = s.gaussian_spinor(dims)[0].numpy()
    return U, phi, 0.12


def test_force_grad_matches_dense_fd(tiny):
    """G = dS/dRe U + i dS/dIm U against central differences of the dense action."""
    U, phi, kappa = tiny
    X, Y = _solve_xy(U, phi, kappa, GENERIC)
    G = oracle.force(U, X, Y, kappa, GENERIC, mode=0)
    rng = np.random.default_rng(0)
    eps = 1e-5
    worst = 0.0
    for _ in range(12):
        t, z, y, x = (rng.integers(n) for n in U.shape[:4])
        mu, a, b = rng.integers(4), rng.integers(3), rng.integers(3)
        d = []
        for unit in (1.0, 1j):
            Up, Um = U.copy(), U.copy()
            Up[t, z, y, x, mu, a, b] += eps * unit
            Um[t, z, y, x, mu, a, b] -= eps * unit
            d.append((dense.action(Up, phi, kappa, GENERIC)
                      - dense.action(Um, phi, kappa, GENERIC)) / (2 * eps))
        fd = d[0] + 1j * d[1]
        worst = max(worst, abs(fd - G[t, z, y, x, mu, a, b]))
    assert worst < 1e-6 * np.abs(G).max()


def _random_su3_generator(rng):
    h = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    h = 0.5 * (h + h.conj().T)
    return h - np.trace(h) / 3 * np.eye(3)


def test_force_lie_matches_dense_fd(tiny):
    """dS/de for U_mu(x) -> exp(i e H) U_mu(x) equals Tr(H F); F Hermitian, traceless."""
    U, phi, kappa = tiny
    X, Y = _solve_xy(U, phi, kappa, GENERIC)
    F = oracle.force(U, X, Y, kappa, GENERIC, mode=1)
    assert np.abs(F - F.conj().swapaxes(-1, -2)).max() < 1e-13
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13
    rng = np.random.default_rng(1)
    eps = 1e-5
    for _ in range(8):
        site = tuple(int(rng.integers(n)) for n in U.shape[:4])
        mu = int(rng.integers(4))
        H = _random_su3_generator(rng)
        vals = []
        for sgn in (1, -1):
            Ue = U.copy()
            Ue[site + (mu,)] = expm(1j * sgn * eps * H) @ U[site + (mu,)]
            vals.append(dense.action(Ue, phi, kappa, GENERIC))
        fd = (vals[0] - vals[1]) / (2 * eps)
        pred = np.trace(H @ F[site + (mu,)]).real
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))


def test_force_identities_phi_from_eta():
    """phi = M^H eta gives Y = M X = eta and S = phi^H X = |eta|^2."""
    dims = (4, 2, 2, 4)
    s = Synth(42)
    U = s.gauge(dims).numpy()
    eta = s.gaussian_spinor(dims)[0].numpy()
    kappa = 0.12
    phi = oracle.apply_M(U, eta, kappa, ANTIPERIODIC, dagger=True)
    X, Y = _solve_xy(U, phi, kappa, ANTIPERIODIC)
    assert rel(Y, eta) < 1e-11
    S = np.vdot(phi, X).real
    assert abs(S - np.vdot(eta, eta).real) < 1e-11 * S


def test_force_gauge_covariance():
    dims = (4, 2, 2, 4)
    s = Synth(43)
    U = s.gauge(dims).numpy()
    X = s.gaussian_spinor(dims)[0].numpy()
    Y = s.gaussian_spinor(dims)[0].numpy()
    G = s.haar_field(dims).numpy()
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    XG = np.einsum("...ab,...sb->...sa", G, X)
    YG = np.einsum("...ab,...sb->...sa", G, Y)
    F = oracle.force(U, X, Y, 0.12, ANTIPERIODIC, mode=1)
    FG = oracle.force(UG, XG, YG, 0.12, ANTIPERIODIC, mode=1)
    expect = G[..., None, :, :] @ F @ G[..., None, :, :].conj().swapaxes(-1, -2)
    assert rel(FG, expect) < 1e-13


def test_local_resolvent_difference_is_exact(tiny):
    """Delta S = S(U') - S(U) = -[(dM X')^H Y + Y'^H (dM X)] with Y = M X, Y' = M' X'
    (exact in dM), checked against dense actions; it is the finite-difference form
    used at full size, where S itself is too large to difference in FP64."""
    U, phi, kappa = tiny
    M = dense.wilson_matrix(U, kappa, GENERIC)
    X = np.linalg.solve(M.conj().T @ M, dense.to_vec(phi))
    Y = M @ X
    rng = np.random.default_rng(3)
    Up = U.copy()
    idx = (1, 0, 1, 0, 2)
    h = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    Up[idx] = expm(0.05j * (h + h.conj().T)) @ U[idx]
    Mp = dense.wilson_matrix(Up, kappa, GENERIC)
    Xp = np.linalg.solve(Mp.conj().T @ Mp, dense.to_vec(phi))
    Yp = Mp @ Xp
    dM = Mp - M
    dS = -(np.vdot(dM @ Xp, Y) + np.vdot(Yp, dM @ X)).real
    direct = dense.action(Up, phi, kappa, GENERIC) - dense.action(U, phi, kappa, GENERIC)
    assert abs(dS - direct) < 1e-10 * abs(direct)
