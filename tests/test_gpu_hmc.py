"""GPU HMC kernels and the trajectory driver against the HMC oracle (through the C ABI).

Gauge force, plaquette action, link exponential and momentum step agree with the
oracle to rounding (FP64); whole leapfrog trajectories, with and without the
pseudofermion, reproduce the oracle's U, P and H to the CG tolerance; flipping
P and integrating back returns the start (reversibility).
"""
import numpy as np
import pytest
import torch

from oracle import hmc
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

DIMS = (4, 4, 4, 6)
ANTI = bc_phases((0, 0, 0, np.pi))
BETA = 5.5


@pytest.fixture(scope="module")
def inputs():
    s = Synth(77)
    U = s.gauge(DIMS, mix=0.5).numpy()
    P = s.momenta(DIMS).numpy()
    Q = s.momenta(DIMS).numpy()
    phi = s.gaussian_spinor(DIMS).numpy()[0]
    return U, P, Q, phi


def _lat(kappa=0.12, csw=0.0):
    return cola.Lattice(DIMS, kappa, ANTI, csw)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_gauge_force_and_action(inputs):
    U, P, Q, phi = inputs
    lat = _lat()
    F = lat.gauge_force(_cuda(U), BETA).cpu().numpy()
    want = hmc.gauge_force(U, BETA)
    assert np.abs(F - want).max() <= 1e-13 * np.abs(want).max()
    S = lat.gauge_action(_cuda(U), BETA)
    assert S == pytest.approx(hmc.gauge_action(U, BETA), rel=1e-13)


@pytest.mark.parametrize("eps", [0.05, 0.7, 3.0])
def test_link_update(inputs, eps):
    """Small steps take the plain series, large ones the scaling-and-squaring path."""
    U, P, Q, phi = inputs
    lat = _lat()
    Ud = _cuda(U)
    lat.link_update(Ud, _cuda(P), eps)
    want = np.einsum("...ij,...jk->...ik", hmc.expi(P, eps), U)
    assert np.abs(Ud.cpu().numpy() - want).max() < 1e-13


def test_momentum_update(inputs):
    U, P, Q, phi = inputs
    lat = _lat()
    F1 = hmc.gauge_force(U, BETA)
    Pd = _cuda(P)
    lat.momentum_update(Pd, _cuda(F1), 0.3, _cuda(Q))
    np.testing.assert_allclose(Pd.cpu().numpy(), P - 0.3 * (F1 + Q), rtol=0, atol=1e-14)


@pytest.mark.parametrize("fermions,integrator", [(False, "leapfrog"), (True, "leapfrog"),
                                                 ("eo", "leapfrog"), (False, "omelyan"),
                                                 ("eo", "omelyan"), ("eo", "leapfrog_mts"),
                                                 (False, "leapfrog_mts")])
def test_trajectory_matches_oracle(inputs, fermions, integrator):
    """fermions: none, the full-lattice pseudofermion, or the even-odd one."""
    U, P, Q, phi = inputs
    lat = _lat()
    eo = fermions == "eo"
    kw = dict(phi=phi, kappa=0.12, bc=ANTI, tol=1e-13, eo=eo) if fermions else {}
    U1, P1, H0, H1 = hmc.trajectory(U, P, BETA, 0.05, 5, integrator=integrator, n_gauge=3,
                                    **kw)
    Ud, Pd = _cuda(U), _cuda(P)
    info = lat.hmc_trajectory(Ud, Pd, BETA, 0.05, 5, phi=_cuda(phi) if fermions else None,
                              cg_tol=1e-13, eo=eo, integrator=integrator, n_gauge=3)
    assert info["status"] == cola.COLA_OK, info
    assert np.abs(Ud.cpu().numpy() - U1).max() < 1e-10
    assert np.abs(Pd.cpu().numpy() - P1).max() < 1e-9
    assert info["H0"] == pytest.approx(H0, rel=1e-11)
    assert info["H1"] == pytest.approx(H1, rel=1e-11)
    assert info["dH"] == pytest.approx(H1 - H0, abs=1e-7)
    assert (info["cg_iterations"] > 0) == bool(fermions)


@pytest.mark.parametrize("scheme", ["FP32_RELIABLE", "FP16_DEFECT"])
def test_trajectory_mixed_precision_solves(inputs, scheme):
    """The fermion solves in mixed precision (FP64 true residual to cg_tol) give the
    FP64 oracle's trajectory to the solver tolerance."""
    U, P, Q, phi = inputs
    lat = _lat()
    U1, P1, H0, H1 = hmc.trajectory(U, P, BETA, 0.05, 4, phi=phi, kappa=0.12, bc=ANTI,
                                    tol=1e-13, eo=True, integrator="omelyan")
    Ud, Pd = _cuda(U), _cuda(P)
    info = lat.hmc_trajectory(Ud, Pd, BETA, 0.05, 4, phi=_cuda(phi), cg_tol=1e-12, eo=True,
                              integrator="omelyan",
                              cg_scheme=getattr(cola, "COLA_CG_" + scheme))
    assert info["status"] == cola.COLA_OK, info
    assert np.abs(Ud.cpu().numpy() - U1).max() < 1e-9
    assert np.abs(Pd.cpu().numpy() - P1).max() < 1e-8
    assert info["dH"] == pytest.approx(H1 - H0, abs=1e-6)


def test_single_step_trajectory_and_momentum_without_second_force(inputs):
    """nsteps = 1 (half step, one link step, half step) and P -= eps F1 with F2 absent."""
    U, P, Q, phi = inputs
    lat = _lat()
    U1, P1, H0, H1 = hmc.trajectory(U, P, BETA, 0.1, 1)
    Ud, Pd = _cuda(U), _cuda(P)
    info = lat.hmc_trajectory(Ud, Pd, BETA, 0.1, 1)
    assert np.abs(Ud.cpu().numpy() - U1).max() < 1e-12
    assert info["dH"] == pytest.approx(H1 - H0, abs=1e-8)
    Pd = _cuda(P)
    lat.momentum_update(Pd, _cuda(Q), 0.5)
    np.testing.assert_allclose(Pd.cpu().numpy(), P - 0.5 * Q, rtol=0, atol=1e-15)


@pytest.mark.parametrize("eo,integrator", [(False, "leapfrog"), (True, "leapfrog"),
                                            (True, "omelyan"), (True, "leapfrog_mts")])
def test_trajectory_reversible(inputs, eo, integrator):
    U, P, Q, phi = inputs
    lat = _lat()
    Ud, Pd = _cuda(U), _cuda(P)
    a = lat.hmc_trajectory(Ud, Pd, BETA, 0.05, 6, phi=_cuda(phi), cg_tol=1e-14, eo=eo,
                           integrator=integrator, n_gauge=3)
    Pd.neg_()
    b = lat.hmc_trajectory(Ud, Pd, BETA, 0.05, 6, phi=_cuda(phi), cg_tol=1e-14, eo=eo,
                           integrator=integrator, n_gauge=3)
    assert np.abs(Ud.cpu().numpy() - U).max() < 1e-10
    assert np.abs(Pd.cpu().numpy() + P).max() < 1e-9
    assert a["dH"] + b["dH"] == pytest.approx(0.0, abs=1e-8)


def test_trajectory_argument_errors(inputs):
    U, P, Q, phi = inputs
    lat = _lat()
    with pytest.raises(cola.ColaError):
        lat.hmc_trajectory(_cuda(U), _cuda(P), BETA, 0.05, 0)
    with pytest.raises(cola.ColaError):
        lat.hmc_trajectory(_cuda(U), _cuda(P), BETA, -0.1, 3)
    with pytest.raises(cola.ColaError):
        lat.hmc_trajectory(_cuda(U), _cuda(P), BETA, 0.05, 3, integrator="leapfrog_mts",
                           n_gauge=0)
    clover = _lat(kappa=0.118, csw=1.0)
    with pytest.raises(cola.ColaError):
        clover.hmc_trajectory(_cuda(U), _cuda(P), BETA, 0.05, 3, phi=_cuda(phi))


def test_quenched_sampler_reaches_the_known_plaquette():
    """End to end: pure-gauge HMC (Omelyan, Metropolis with seeded draws) on 4^4 at
    beta = 6.0 from a cold start; <exp(-dH)> = 1 within errors and the plaquette in the
    range of this action's known value there (about 0.594 in large volume; 4^4 sits a
    little above it)."""
    from paper_2302_00850_amd.synth import unit_gauge
    dims = (4, 4, 4, 4)
    beta = 6.0
    s = Synth(21, device="cuda", rng="torch")
    rng = np.random.default_rng(21)
    lat = cola.Lattice(dims, 0.12, ANTI, 0.0)
    U = unit_gauge(dims, device="cuda")
    V = int(np.prod(dims))
    plaq, w = [], []
    for k in range(300):
        P = s.momenta(dims)
        U0 = U.clone()
        info = lat.hmc_trajectory(U, P, beta, 0.05, 20, integrator="omelyan")
        if not (k < 50 or rng.random() < np.exp(min(0.0, -info["dH"]))):
            U.copy_(U0)
        if k >= 100:
            w.append(np.exp(-info["dH"]))
            plaq.append(1.0 - lat.gauge_action(U, beta) / (beta * 6 * V))
    assert abs(np.mean(w) - 1.0) < 0.05
    assert 0.58 < np.mean(plaq) < 0.63


def test_long_run_links_stay_su3():
    """250 even-odd Omelyan trajectories with FP32 reliable-update solves (momenta
    refreshed each time, every trajectory kept): the link update re-unitarises, so the
    field still passes the SU(3) check that the mixed-precision solves require, and the
    next trajectory from the evolved field is still the oracle's."""
    dims = (4, 4, 4, 4)
    s = Synth(91)
    U = s.gauge(dims, mix=0.5)
    phi = s.gaussian_spinor(dims)[0]
    lat = cola.Lattice(dims, 0.12, ANTI)
    Ud, phid = U.cuda(), phi.cuda()
    for k in range(250):
        Pd = s.momenta(dims).cuda()
        info = lat.hmc_trajectory(Ud, Pd, BETA, 0.1, 4, phi=phid, cg_tol=1e-10, eo=True,
                                  integrator="omelyan", cg_scheme=cola.COLA_CG_FP32_RELIABLE)
        assert info["status"] == cola.COLA_OK, (k, info)
    Uh = Ud.cpu().numpy()
    dev = np.abs(np.einsum("...ij,...kj->...ik", Uh, Uh.conj()) - np.eye(3)).max()
    assert dev < 1e-13, dev
    assert np.abs(np.linalg.det(Uh) - 1).max() < 1e-13
    lat.set_gauge(Ud)
    assert lat.gauge_is_su3
    P = s.momenta(dims).numpy()
    U1, P1, H0, H1 = hmc.trajectory(Uh, P, BETA, 0.1, 4, phi=phi.numpy(), kappa=0.12, bc=ANTI,
                                    tol=1e-13, eo=True, integrator="omelyan")
    Pd = _cuda(P)
    info = lat.hmc_trajectory(Ud, Pd, BETA, 0.1, 4, phi=phid, cg_tol=1e-13, eo=True,
                              integrator="omelyan")
    assert info["status"] == cola.COLA_OK
    assert np.abs(Ud.cpu().numpy() - U1).max() < 1e-10
    assert info["dH"] == pytest.approx(H1 - H0, abs=1e-7)
