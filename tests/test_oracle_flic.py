"""Pins of the FLIC oracle: APE smearing and the fat-link irrelevant clover operator.

Operator: with F = U it is the Wilson-clover operator of the C oracle; the dense matrix
assembled from the pinned dense hopping matrices (naive part of U, Wilson term of F) on a
lattice with extent-2 directions; the dagger form is the adjoint; gauge covariance with
both fields transformed.  Smearing: alpha = 0 and U = 1 are fixed points, a pure gauge
stays pure gauge, smearing commutes with gauge transformations, the result is SU(3) and
smoother (larger plaquette).
"""
import numpy as np
import pytest

import oracle
from oracle import dense, flic
from paper_2302_00850_amd.synth import Synth, bc_phases, unit_gauge
from tests._util import g5, rel

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))


def _gauge_transform(U, G):
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    return UG


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_flic_with_thin_fat_links_is_wilson_clover(csw):
    dims = (4, 4, 2, 4)
    s = Synth(81)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims).numpy()[0]
    A = oracle.clover(U, 0.118, csw) if csw else None
    want = oracle.apply_M(U, psi, 0.118, GENERIC, clover=A)
    got = flic.apply_flic(U, U, psi, 0.118, GENERIC, csw)
    assert rel(got, want) < 1e-14


def test_flic_hop_matches_dense_assembly():
    """D_FLIC = R(F) + N(U): the Wilson-term part R(W) = (H + g5 H g5) / 2 and the naive part
    N(W) = (H - g5 H g5) / 2 of the dense hopping matrix H(W), on 2x2x2x4."""
    dims = (2, 2, 2, 4)
    s = Synth(82)
    U = s.gauge(dims, mix=0.6).numpy()
    F = flic.ape_smear(U, 0.7, 2)
    psi = s.gaussian_spinor(dims).numpy()[0]
    G5 = np.kron(np.eye(int(np.prod(dims))), np.kron(dense.gamma5(), np.eye(3)))
    HF, HU = dense.hop_matrix(F, GENERIC), dense.hop_matrix(U, GENERIC)
    D = 0.5 * (HF + G5 @ HF @ G5) + 0.5 * (HU - G5 @ HU @ G5)
    want = D @ dense.to_vec(psi)
    got = dense.to_vec(flic.flic_hop(U, F, psi, GENERIC))
    assert rel(got, want) < 1e-14
    # and F really differs from U here
    assert rel(F, U) > 1e-2


def test_flic_dagger_is_the_adjoint_and_gauge_covariant():
    dims = (4, 2, 4, 4)
    s = Synth(83)
    U = s.gauge(dims).numpy()
    F = flic.ape_smear(U, 0.7, 4)
    psi = s.gaussian_spinor(dims).numpy()[0]
    eta = s.gaussian_spinor(dims).numpy()[0]
    kappa, csw = 0.12, 1.0
    lhs = np.vdot(eta, flic.apply_flic(U, F, psi, kappa, GENERIC, csw))
    rhs = np.vdot(flic.apply_flic(U, F, eta, kappa, GENERIC, csw, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    G = s.haar_field(dims).numpy()
    UG, FG = _gauge_transform(U, G), _gauge_transform(F, G)
    Gpsi = np.einsum("...ab,...sb->...sa", G, psi)
    got = flic.apply_flic(UG, FG, Gpsi, kappa, GENERIC, csw)
    want = np.einsum("...ab,...sb->...sa", G, flic.apply_flic(U, F, psi, kappa, GENERIC, csw))
    assert rel(got, want) < 1e-13


def test_ape_smearing_fixed_points_and_covariance():
    dims = (4, 4, 2, 4)
    s = Synth(84)
    U = s.gauge(dims).numpy()
    assert np.abs(flic.ape_smear(U, 0.0, 3) - U).max() < 1e-14
    one = unit_gauge(dims).numpy()
    assert np.abs(flic.ape_smear(one, 0.7, 2) - one).max() < 1e-14
    G = s.haar_field(dims).numpy()
    pure = _gauge_transform(one, G)
    assert np.abs(flic.ape_smear(pure, 0.7, 2) - pure).max() < 1e-13
    F = flic.ape_smear(U, 0.7, 3)
    FG = flic.ape_smear(_gauge_transform(U, G), 0.7, 3)
    assert np.abs(FG - _gauge_transform(F, G)).max() < 1e-13
    assert np.abs(F @ F.conj().swapaxes(-1, -2) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(F) - 1).max() < 1e-14
    assert oracle.plaquette(F) > oracle.plaquette(U) + 0.05
