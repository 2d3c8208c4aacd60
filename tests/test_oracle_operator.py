"""Pins of the FP64 oracle's Wilson-Dirac operator against facts that do not
come from the oracle itself: the Clifford algebra, the free-field symbol
1 - kappa sum_mu (2 cos p_mu - 2i g_mu sin p_mu), gamma5-hermiticity, gauge and
translation covariance, and a dense brute-force assembly on tiny lattices."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2302_00850_amd.synth import Synth, bc_phases, unit_gauge
from tests._util import dims_of, g5, rel

ANTIPERIODIC = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))


@pytest.mark.parametrize("table", ["oracle", "dense"])
def test_gamma_table_clifford(table):
    g = [oracle.gamma(mu) for mu in range(4)] if table == "oracle" else dense.gammas()
    for mu, nu in itertools.product(range(4), repeat=2):
        anti = g[mu] @ g[nu] + g[nu] @ g[mu]
        np.testing.assert_allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=0)
    for m in g:
        np.testing.assert_allclose(m, m.conj().T, atol=0)
    g5m = g[0] @ g[1] @ g[2] @ g[3]
    np.testing.assert_allclose(g5m, np.diag([1, 1, -1, -1]), atol=0)
    # (1 -+ g_mu) are rank-2 projectors times 2
    for m in g:
        assert np.linalg.matrix_rank(np.eye(4) - m) == 2


def _plane_wave(dims, n, theta, u):
    lx, ly, lz, lt = dims
    p = [(2 * np.pi * n[mu] + theta[mu]) / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u, np.array(p), ph


@pytest.mark.parametrize("theta", [(0, 0, 0, np.pi), (0.3, -0.5, 0.7, np.pi)])
def test_free_field_symbol(theta):
    """U = 1: M e^{ipx} u = e^{ipx} (a + i sum_mu b_mu g_mu) u with
    a = 1 - 2 kappa sum cos p, b_mu = 2 kappa sin p_mu, p_mu = (2 pi n_mu + theta_mu)/L_mu."""
    dims = (4, 4, 2, 6)
    kappa = 0.12
    U = unit_gauge(dims).numpy()
    bc = bc_phases(theta)
    rng = np.random.default_rng(5)
    gam = dense.gammas()
    for n in [(0, 0, 0, 0), (1, 0, 1, 2), (3, 2, 1, 5), (2, 3, 0, 1)]:
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p, ph = _plane_wave(dims, n, theta, u)
        out = oracle.apply_M(U, psi, kappa, bc)
        a = 1 - 2 * kappa * np.cos(p).sum()
        b = 2 * kappa * np.sin(p)
        symbol = a * np.eye(4) + 1j * sum(b[mu] * gam[mu] for mu in range(4))
        expect = ph[..., None, None] * (symbol @ u)
        assert rel(out, expect) < 1e-14


def test_free_field_eigenvalues_basis_free():
    """The 12x12 momentum block of M has eigenvalues a +- i|b|, six of each
    (checked without any gamma table: the block is read off the oracle)."""
    dims = (4, 2, 4, 8)
    kappa = 0.12
    theta = (0, 0, 0, np.pi)
    U = unit_gauge(dims).numpy()
    for n in [(1, 1, 0, 3), (0, 0, 2, 0)]:
        K = np.zeros((12, 12), dtype=complex)
        for j in range(12):
            u = np.zeros(12, dtype=complex)
            u[j] = 1
            psi, p, ph = _plane_wave(dims, n, theta, u.reshape(4, 3))
            out = oracle.apply_M(U, psi, kappa, ANTIPERIODIC)
            K[:, j] = (out[1, 1, 1, 1] / ph[1, 1, 1, 1]).reshape(12)
        a = 1 - 2 * kappa * np.cos(p).sum()
        bn = np.linalg.norm(2 * kappa * np.sin(p))
        ev = np.linalg.eigvals(K)
        np.testing.assert_allclose(ev.real, a, atol=1e-12)
        np.testing.assert_allclose(np.sort(ev.imag), [-bn] * 6 + [bn] * 6, atol=1e-12)
        # M^H M acts as the scalar a^2 + |b|^2 on the plane wave
        psi, p, ph = _plane_wave(dims, n, theta, np.ones((4, 3)))
        mm = oracle.apply_M(U, oracle.apply_M(U, psi, kappa, ANTIPERIODIC), kappa, ANTIPERIODIC,
                            dagger=True)
        assert rel(mm, (a * a + bn * bn) * psi) < 1e-14


@pytest.mark.parametrize("bc", [ANTIPERIODIC, GENERIC])
def test_gamma5_hermiticity(bc):
    dims = (4, 2, 2, 4)
    s = Synth(11)
    U = s.gauge(dims).numpy()
    eta = s.gaussian_spinor(dims)[0].numpy()
    psi = s.gaussian_spinor(dims)[0].numpy()
    kappa = 0.12
    Mpsi = oracle.apply_M(U, psi, kappa, bc)
    Mdag_eta = oracle.apply_M(U, eta, kappa, bc, dagger=True)
    lhs = np.vdot(eta, Mpsi)
    rhs = np.vdot(Mdag_eta, psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # M^H = g5 M g5
    assert rel(Mdag_eta, g5(oracle.apply_M(U, g5(eta), kappa, bc))) < 1e-15


def _gauge_transform(U, psi, G):
    """U^G_mu(x) = G(x) U_mu(x) G(x+mu)^H, psi^G = G psi."""
    UG = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu  # array axes are (t, z, y, x)
        Gf = np.roll(G, -1, axis=axis)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    return UG, np.einsum("...ab,...sb->...sa", G, psi)


@pytest.mark.parametrize("bc", [ANTIPERIODIC, GENERIC])
def test_gauge_covariance(bc):
    dims = (4, 4, 2, 4)
    s = Synth(3)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims)[0].numpy()
    G = s.haar_field(dims).numpy()
    UG, psiG = _gauge_transform(U, psi, G)
    kappa = 0.137
    for dag in (False, True):
        out = oracle.apply_M(U, psi, kappa, bc, dagger=dag)
        outG = oracle.apply_M(UG, psiG, kappa, bc, dagger=dag)
        assert rel(outG, np.einsum("...ab,...sb->...sa", G, out)) < 1e-14


def _translate(f, mu, theta, is_spinor):
    """Shift a field by one site along +mu; a spinor picks up exp(-i theta) where it
    wraps (the field is e^{i theta}-periodic), links are plain periodic."""
    axis = 3 - mu + (0 if not is_spinor else 0)
    g = np.roll(f, 1, axis=axis)
    if is_spinor:
        idx = [slice(None)] * g.ndim
        idx[axis] = 0
        g[tuple(idx)] *= np.exp(-1j * theta[mu])
    return g


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_translation_covariance(mu):
    theta = (0.3, -0.5, 0.7, np.pi)
    bc = bc_phases(theta)
    dims = (4, 2, 4, 4)
    s = Synth(21)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims)[0].numpy()
    kappa = 0.11
    out = oracle.apply_M(U, psi, kappa, bc)
    Ut = _translate(U, mu, theta, False)
    psit = _translate(psi, mu, theta, True)
    out_t = oracle.apply_M(Ut, psit, kappa, bc)
    assert rel(out_t, _translate(out, mu, theta, True)) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 2)])
def test_dense_assembly_matches_stencil(dims):
    s = Synth(7)
    U = s.gauge(dims).numpy()
    kappa = 0.12
    M = dense.wilson_matrix(U, kappa, GENERIC)
    for dag in (False, True):
        Mm = M.conj().T if dag else M
        for _ in range(3):
            psi = s.gaussian_spinor(dims)[0].numpy()
            out = oracle.apply_M(U, psi, kappa, GENERIC, dagger=dag)
            assert rel(dense.to_vec(out), Mm @ dense.to_vec(psi)) < 1e-14


def test_dense_assembly_with_clover():
    dims = (2, 2, 2, 4)
    s = Synth(8)
    U = s.gauge(dims).numpy()
    kappa, csw = 0.118, 1.0
    A = oracle.clover(U, kappa, csw)
    M = dense.wilson_matrix(U, kappa, ANTIPERIODIC, clover=A)
    psi = s.gaussian_spinor(dims)[0].numpy()
    out = oracle.apply_M(U, psi, kappa, ANTIPERIODIC, clover=A)
    assert rel(dense.to_vec(out), M @ dense.to_vec(psi)) < 1e-14
    out = oracle.apply_M(U, psi, kappa, ANTIPERIODIC, clover=A, dagger=True)
    assert rel(dense.to_vec(out), M.conj().T @ dense.to_vec(psi)) < 1e-14


@pytest.mark.parametrize("with_clover", [False, True])
def test_schur_complement_matches_dense(with_clover):
    dims = (2, 2, 2, 4)
    s = Synth(9)
    U = s.gauge(dims).numpy()
    kappa = 0.12
    A = oracle.clover(U, kappa, 1.0) if with_clover else None
    Ai = oracle.site_inverse(A) if with_clover else None
    M = dense.wilson_matrix(U, kappa, GENERIC, clover=A)
    S = dense.schur_matrix(M, dims)
    even = dense.parity_vector(dims) == 0
    psi = s.gaussian_spinor(dims)[0].numpy()
    for dag in (False, True):
        out = oracle.apply_schur(U, psi, kappa, GENERIC, clover=A, clover_inv=Ai, dagger=dag)
        v = dense.to_vec(out)
        Sm = S.conj().T if dag else S
        assert rel(v[even], Sm @ dense.to_vec(psi)[even]) < 1e-13
        assert np.all(v[~even] == 0)


def test_hop_degenerate_extent_two_adds_both_neighbours():
    """On an extent-2 direction x+mu = x-mu: the two hops must add, not overwrite."""
    dims = (2, 2, 2, 2)
    U = unit_gauge(dims).numpy()
    psi = np.zeros((2, 2, 2, 2, 4, 3), dtype=complex)
    psi[0, 0, 0, 1, 0, 0] = 1.0  # a single entry at x = 1
    out = oracle.hop(U, psi, bc_phases((0, 0, 0, 0)))
    # site x = 0 receives (1 - g_x) e_0 + (1 + g_x) e_0 = 2 e_0 from the two x-hops
    np.testing.assert_allclose(out[0, 0, 0, 0, :, 0], [2, 0, 0, 0], atol=1e-15)
