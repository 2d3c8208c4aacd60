"""GPU multi-shift CG against the multi-shift oracle (through the C ABI): every shifted
solution, the shared iteration count and the true residuals, on the full-lattice and
even-odd systems, with and without clover; argument errors."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multishift
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

DIMS = (6, 4, 4, 10)
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
SHIFTS = [0.0, 0.004, 0.02, 0.1, 0.3, 0.9, 1.7, 4.0]


@pytest.fixture(scope="module")
def fields():
    s = Synth(303)
    return s.gauge(DIMS).numpy(), s.gaussian_spinor(DIMS).numpy()[0]


@pytest.mark.parametrize("system", [0, 1])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_multishift_matches_oracle(fields, system, csw):
    U, b = fields
    kappa = 0.118 if csw else 0.12
    A = oracle.clover(U, kappa, csw) if csw else None
    Ai = oracle.site_inverse(A) if csw else None
    tol = 1e-10
    want, n_or = multishift.multishift_cg(U, b, SHIFTS, kappa, GENERIC, system=system, tol=tol,
                                          clover=A, clover_inv=Ai)
    lat = cola.Lattice(DIMS, kappa, GENERIC, csw)
    lat.set_gauge(torch.from_numpy(U).cuda())
    sysid = cola.COLA_SYS_MDAGM if system == 0 else cola.COLA_SYS_SCHUR
    x, info = lat.cg_multishift(torch.from_numpy(b).cuda(), SHIFTS, system=sysid, tol=tol)
    assert info["status"] == cola.COLA_OK, info
    assert abs(info["iterations"] - n_or) <= 1
    xs = x.cpu().numpy()
    be = b if system == 0 else np.where(oracle.parity_mask(DIMS)[..., None, None], b, 0)
    for q, sig in enumerate(SHIFTS):
        assert rel(xs[q], want[q]) < 1e-7, sig
        res = be - multishift.apply_A(U, xs[q], kappa, GENERIC, system, A, Ai) - sig * xs[q]
        r = np.linalg.norm(res) / np.linalg.norm(be)
        assert r <= 2 * tol, (sig, r)
        assert info["true_rel_residual"][q] == pytest.approx(r, rel=1e-3, abs=1e-14)
    if system == 1:
        assert np.all(np.where(oracle.parity_mask(DIMS)[..., None, None], 0, xs) == 0)


@pytest.mark.parametrize("shifts", [[0.25], list(np.geomspace(1e-3, 10.0, 16))])
def test_multishift_single_and_sixteen_shifts(fields, shifts):
    """One shift (no unshifted member) and the maximum of sixteen."""
    U, b = fields
    tol = 1e-10
    want, n_or = multishift.multishift_cg(U, b, shifts, 0.12, GENERIC, system=1, tol=tol)
    lat = cola.Lattice(DIMS, 0.12, GENERIC)
    lat.set_gauge(torch.from_numpy(U).cuda())
    x, info = lat.cg_multishift(torch.from_numpy(b).cuda(), shifts, system=cola.COLA_SYS_SCHUR,
                                tol=tol)
    assert info["status"] == cola.COLA_OK, info
    assert abs(info["iterations"] - n_or) <= 1
    xs = x.cpu().numpy()
    for q in range(len(shifts)):
        assert rel(xs[q], want[q]) < 1e-7
        assert info["true_rel_residual"][q] <= 2 * tol


def test_multishift_argument_errors(fields):
    U, b = fields
    lat = cola.Lattice(DIMS, 0.12, GENERIC)
    lat.set_gauge(torch.from_numpy(U).cuda())
    bd = torch.from_numpy(b).cuda()
    for shifts in ([], [-0.1, 0.2], [0.1] * 17):
        with pytest.raises(cola.ColaError):
            lat.cg_multishift(bd, shifts)
    with pytest.raises(cola.ColaError):
        lat.cg_multishift(bd, [0.1], system=cola.COLA_SYS_PROPAGATOR)
