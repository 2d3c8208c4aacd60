"""Pins of the oracle's site-sampled operator and its plaquette.

`oracle.apply_M_sites` assembles the clover matrix of each requested site on
its own (it is the checker of the full-size GPU tests, where the whole-lattice
clover field does not fit the host), so it is compared here, at every site of a
small lattice with an extent-2 direction and generic boundary phases, against
`oracle.apply_M` fed the whole-lattice `oracle.clover` field -- two routes that
share only the gamma table.  `oracle.plaquette` is pinned by U = 1, the closed
form of a constant abelian flux in each plane, gauge invariance, and the
numpy plaquette action of the HMC oracle (itself pinned by finite differences
and closed forms)."""
import numpy as np
import pytest

import oracle
from oracle import hmc
from paper_2302_00850_amd.synth import Synth, bc_phases, unit_gauge
from tests._util import rel

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))


@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_M_sites_matches_whole_lattice_operator(csw, dagger):
    dims = (4, 4, 2, 4)
    kappa = 0.118
    s = Synth(41)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims).numpy()[0]
    V = int(np.prod(dims))
    got = oracle.apply_M_sites(U, psi, kappa, GENERIC, np.arange(V), csw=csw, dagger=dagger)
    A = oracle.clover(U, kappa, csw) if csw else None
    ref = oracle.apply_M(U, psi, kappa, GENERIC, clover=A, dagger=dagger).reshape(V, 4, 3)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    # the sampled form at a scattered subset (order and repeats do not matter)
    sub = np.array([V - 1, 0, 17, 17, 5])
    part = oracle.apply_M_sites(U, psi, kappa, GENERIC, sub, csw=csw, dagger=dagger)
    assert np.array_equal(part, got[sub])


def test_apply_M_sites_clover_term_is_not_trivial():
    """Guard on the pin above: with these fields the clover term moves M by far more
    than the 1e-14 tolerance, so a dropped or mis-signed clover term would fail it."""
    dims = (4, 4, 2, 4)
    s = Synth(41)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims).numpy()[0]
    V = int(np.prod(dims))
    m0 = oracle.apply_M_sites(U, psi, 0.118, GENERIC, np.arange(V), csw=0.0)
    m1 = oracle.apply_M_sites(U, psi, 0.118, GENERIC, np.arange(V), csw=1.0)
    assert rel(m1, m0) > 1e-3


def _constant_flux_gauge(dims, mu, nu):
    """One flux quantum of a U(1) field in the (mu, nu) plane, embedded as
    diag(e^{i th}, e^{-i th}, 1): every (mu, nu) plaquette is diag(e^{if}, e^{-if}, 1)
    with f = 2 pi / (L_mu L_nu), every other plaquette is 1."""
    L = dims
    f = 2 * np.pi / (L[mu] * L[nu])
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


def test_plaquette_unit_gauge_is_one():
    assert oracle.plaquette(unit_gauge((4, 2, 2, 4)).numpy()) == 1.0


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 3), (1, 2), (2, 3)])
def test_plaquette_constant_abelian_flux(mu, nu):
    dims = (4, 6, 2, 4)
    U, f = _constant_flux_gauge(dims, mu, nu)
    # one plane of six has Re Tr / 3 = (1 + 2 cos f) / 3, the other five 1
    expect = (5.0 + (1.0 + 2.0 * np.cos(f)) / 3.0) / 6.0
    assert abs(oracle.plaquette(U) - expect) < 1e-14


def test_plaquette_gauge_invariant_and_equals_the_action():
    dims = (4, 4, 2, 4)
    s = Synth(42)
    U = s.gauge(dims).numpy()
    G = s.haar_field(dims).numpy()
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ Gf.conj().swapaxes(-1, -2)
    p = oracle.plaquette(U)
    assert abs(oracle.plaquette(UG) - p) < 1e-14
    V = int(np.prod(dims))
    beta = 5.6
    assert abs(p - (1.0 - hmc.gauge_action(U, beta) / (6 * V * beta))) < 1e-14
    # the mixed generator field sits well below 1 (so the comparison is not trivial)
    assert 0.5 < p < 0.95


@pytest.mark.parametrize("dagger", [False, True])
def test_hop_sites_matches_whole_lattice_hop(dagger):
    dims = (4, 2, 4, 4)
    s = Synth(43)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims).numpy()[0]
    V = int(np.prod(dims))
    got = oracle.hop_sites(U, psi, GENERIC, np.arange(V), dagger=dagger)
    ref = oracle.hop(U, psi, GENERIC, dagger=dagger).reshape(V, 4, 3)
    assert np.array_equal(got, ref)
