"""The fat-link irrelevant clover (FLIC) operator on the GPU, through the C ABI.

APE smearing against the oracle's (links to 1e-12); the FLIC operator M and M^H on the
full lattice in FP64 (1e-13) and FP32 (2e-6), 1 and 12 right-hand sides, with and
without the clover term of the smeared field, against the oracle's FLIC operator; the
even-odd machinery on FLIC through the propagator solve M x = b (every scheme), whose
residual the oracle recomputes; the operator returns to Wilson after set_gauge; the
calls that FLIC does not support refuse it.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import flic
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import assert_close, rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
ANTI = bc_phases((0, 0, 0, np.pi))
DIMS = (6, 4, 4, 10)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def fields():
    s = Synth(121)
    U = s.gauge(DIMS, mix=0.5).numpy()
    psi = s.gaussian_spinor(DIMS, 12).numpy()
    F = flic.ape_smear(U, 0.7, 4)
    return U, F, psi


@pytest.mark.parametrize("alpha,n", [(0.7, 1), (0.7, 4), (0.45, 3), (0.0, 2)])
def test_ape_smear_matches_oracle(fields, alpha, n):
    U, _, _ = fields
    lat = cola.Lattice(DIMS, 0.12, ANTI)
    F = lat.ape_smear(_cuda(U), alpha, n).cpu().numpy()
    want = flic.ape_smear(U, alpha, n)
    assert np.abs(F - want).max() < 1e-12
    # in place (F aliasing U) gives the same field
    Ud = _cuda(U)
    cola.cola_ape_smear(lat.h, Ud.data_ptr(), Ud.data_ptr(), alpha, n,
                        torch.cuda.current_stream().cuda_stream)
    assert np.abs(Ud.cpu().numpy() - want).max() < 1e-12


@pytest.mark.parametrize("prec,tol", [(cola.COLA_FP64, 1e-13), (cola.COLA_FP64_12, 1e-13),
                                      (cola.COLA_FP32, 2e-6)])
@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("nrhs", [1, 12])
def test_flic_operator_matches_oracle(fields, prec, tol, csw, nrhs):
    U, F, psi = fields
    kappa = 0.118 if csw else 0.12
    lat = cola.Lattice(DIMS, kappa, GENERIC, csw)
    lat.set_gauge(_cuda(U))
    lat.set_fat_gauge(_cuda(F))
    src = psi[:nrhs]
    pin = lat.pack(_cuda(src), prec, -1)
    src_r = lat.unpack(pin, prec, nrhs, -1).cpu().numpy()
    for op, dag in ((cola.COLA_OP_M, False), (cola.COLA_OP_MDAG, True)):
        out = lat.empty_packed(prec, nrhs, -1)
        lat.dslash(out, pin, op, -1, prec, nrhs)
        got = lat.unpack(out, prec, nrhs, -1).cpu().numpy()
        for q in range(nrhs):
            want = flic.apply_flic(U, F, src_r[q], kappa, GENERIC, csw=csw, dagger=dag)
            assert_close(got[q], want, tol, (prec, csw, nrhs, dag, q))


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP64, cola.COLA_CG_FP32_RELIABLE,
                                    cola.COLA_CG_FP32_DEFECT])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_flic_propagator_solve(fields, scheme, csw):
    """M x = b through the even-odd Schur normal equations of the FLIC operator (the hops
    with every epilogue, the clover blocks of the smeared field): the oracle's FLIC
    operator applied to x gives b back."""
    U, F, psi = fields
    kappa = 0.118 if csw else 0.12
    lat = cola.Lattice(DIMS, kappa, ANTI, csw)
    lat.set_gauge(_cuda(U))
    lat.set_fat_gauge(_cuda(F))
    b = psi[:2]
    x, info = lat.cg(_cuda(b), system=cola.COLA_SYS_PROPAGATOR, scheme=scheme, tol=1e-11)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(2):
        r = rel(flic.apply_flic(U, F, xs[q], kappa, ANTI, csw=csw), b[q])
        assert r <= 1.1e-11, (q, r)  # the full-lattice residual meets tol


def test_flic_block_cg_propagators(fields):
    """Block CG (FP32 inner, FP64 defect correction) on the FLIC propagator system: the
    oracle's FLIC operator applied to x gives b back to the tolerance."""
    U, F, psi = fields
    kappa = 0.118
    lat = cola.Lattice(DIMS, kappa, ANTI, 1.0)
    lat.set_gauge(_cuda(U))
    lat.set_fat_gauge(_cuda(F))
    b = psi[:4]
    x, info = lat.cg(_cuda(b), system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP32_DEFECT,
                     tol=1e-10, block=1)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(4):
        r = rel(flic.apply_flic(U, F, xs[q], kappa, ANTI, csw=1.0), b[q])
        assert r <= 1.1e-10, (q, r)


def test_flic_normal_cg_and_return_to_wilson(fields):
    U, F, psi = fields
    kappa = 0.12
    lat = cola.Lattice(DIMS, kappa, ANTI)
    lat.set_gauge(_cuda(U))
    lat.set_fat_gauge(_cuda(F))
    x, info = lat.cg(_cuda(psi[:1]), system=cola.COLA_SYS_MDAGM, tol=1e-10)
    assert info["status"] == cola.COLA_OK
    xs = x.cpu().numpy()[0]
    Mx = flic.apply_flic(U, F, xs, kappa, ANTI)
    assert rel(flic.apply_flic(U, F, Mx, kappa, ANTI, dagger=True), psi[0]) <= 1.05e-10
    # set_gauge returns the handle to the Wilson operator
    lat.set_gauge(_cuda(U))
    pin = lat.pack(_cuda(psi[:1]), cola.COLA_FP64, -1)
    out = lat.empty_packed(cola.COLA_FP64, 1, -1)
    lat.dslash(out, pin, cola.COLA_OP_M, -1, cola.COLA_FP64, 1)
    got = lat.unpack(out, cola.COLA_FP64, 1, -1).cpu().numpy()[0]
    assert_close(got, oracle.apply_M(U, psi[0], kappa, ANTI), 1e-13)


def test_flic_refusals(fields):
    U, F, psi = fields
    lat = cola.Lattice(DIMS, 0.12, ANTI)
    with pytest.raises(cola.ColaError):
        lat.set_fat_gauge(_cuda(F))  # before set_gauge
    lat.set_gauge(_cuda(U))
    bad = F.copy()
    bad[0, 0, 0, 0, 0] *= 1.01
    with pytest.raises(cola.ColaError):
        lat.set_fat_gauge(_cuda(bad))  # not SU(3)
    lat.set_fat_gauge(_cuda(F))
    pin = lat.pack(_cuda(psi[:1]), cola.COLA_FP16, 1)
    out = lat.empty_packed(cola.COLA_FP16, 1, 0)
    with pytest.raises(cola.ColaError):
        lat.dslash(out, pin, cola.COLA_OP_HOP, 0, cola.COLA_FP16, 1)
    with pytest.raises(cola.ColaError):
        lat.force(_cuda(psi[0]), _cuda(psi[1]))
    Ud = _cuda(U)
    Pd = torch.zeros_like(Ud)
    with pytest.raises(cola.ColaError):
        lat.hmc_trajectory(Ud, Pd, 5.5, 0.1, 1)
