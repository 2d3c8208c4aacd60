"""Low-eigenmode solver and deflated CG on the GPU, through the C ABI.

Eigenpairs of A = M^H M (full lattice) and S^H S (even sites), plain Wilson and
clover, against the oracle's accelerated-CG eigensolver run from the same starting
vectors (eigenvalues to 1e-9 relative, eigenvectors up to a phase) and against a
dense eigendecomposition on a lattice with extent-2 directions; residuals recomputed
by the oracle.  Deflated CG: the oracle-checked residual meets the tolerance, the
iteration count drops below plain CG's, and the solution agrees with the oracle's
deflated CG.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import dense, eigen
from oracle.multishift import apply_A
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

ANTI = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _lat(U, bc, kappa, csw=0.0):
    lat = cola.Lattice(tuple(U.shape[:4][::-1]), kappa, bc, csw)
    lat.set_gauge(torch.from_numpy(U).cuda())
    return lat


def _even(v):
    return np.where(oracle.parity_mask(v.shape[-6:-2][::-1])[..., None, None], v, 0)


def test_eigensolve_matches_oracle():
    """S^H S on 4^4 (a field whose four lowest modes the method separates in about 25
    sweeps): the same converged eigenpairs as the oracle's solver from the same start."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    s = Synth(71)
    U = s.gauge(dims, mix=0.9).numpy()
    X0 = s.gaussian_spinor(dims, 4).numpy()
    lam_o, X_o, sweeps_o, _ = eigen.eigensolve(U, X0, kappa, GENERIC, system=1, tol=1e-10)
    assert sweeps_o < 100
    lat = _lat(U, GENERIC, kappa)
    lam, X, info = lat.eigensolve(_cuda(X0), system=cola.COLA_SYS_SCHUR, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    lam = np.array(lam)
    assert np.all(np.abs(lam - lam_o) <= 1e-9 * lam_o), (lam, lam_o)
    Xg = X.cpu().numpy()
    for i in range(len(lam)):
        v = _even(Xg[i])
        assert np.all(Xg[i] == v)  # odd sites zero
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        # residual recomputed by the oracle
        Av = _even(apply_A(U, v, kappa, GENERIC, 1))
        assert np.linalg.norm(Av - lam[i] * v) <= 2e-10 * lam[i]
        assert info["residuals"][i] <= 1e-10
        # the same eigenvector up to a phase
        assert abs(abs(np.vdot(X_o[i], v)) - 1) < 1e-8, i
    # a sweep budget too small: the current Ritz pairs come back, flagged
    _, _, info2 = lat.eigensolve(_cuda(X0), system=cola.COLA_SYS_SCHUR, tol=1e-10,
                                 max_sweeps=2)
    assert info2["status"] == cola.COLA_NOT_CONVERGED and info2["sweeps"] == 2


@pytest.mark.parametrize("system", [cola.COLA_SYS_MDAGM, cola.COLA_SYS_SCHUR])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_eigensolve_extent2_against_dense(system, csw):
    """2x2x2x4 (extent-2 directions), M^H M and S^H S, plain and clover: the eigenvalues
    are the lowest of the dense normal matrix assembled block by block, and the
    eigenvectors satisfy the dense eigen-equation."""
    dims = (2, 2, 2, 4)
    kappa = 0.11
    s = Synth(72)
    U = s.gauge(dims, mix=0.6).numpy()
    # four modes: the fifth and sixth eigenvalues of M^H M here differ by 0.05%, which the
    # one-vector-at-a-time minimisation resolves only very slowly
    X0 = s.gaussian_spinor(dims, 4).numpy()
    lat = _lat(U, GENERIC, kappa, csw)
    lam, X, info = lat.eigensolve(_cuda(X0), system=system, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    A = oracle.clover(U, kappa, csw) if csw else None
    M = dense.wilson_matrix(U, kappa, GENERIC, clover=A)
    if system == cola.COLA_SYS_MDAGM:
        H = M.conj().T @ M
        rows = np.ones(M.shape[0], dtype=bool)
    else:
        S = dense.schur_matrix(M, dims)
        H = S.conj().T @ S
        rows = dense.parity_vector(dims) == 0
    w = np.linalg.eigvalsh(H)
    assert np.all(np.abs(np.array(lam) - w[:4]) <= 1e-9 * w[:4]), (lam, w[:4])
    Xg = X.cpu().numpy().reshape(4, -1)
    for i in range(4):
        v = Xg[i][rows]
        assert np.linalg.norm(H @ v - lam[i] * v) <= 2e-10 * lam[i]


def test_eigensolve_argument_errors():
    dims = (4, 4, 4, 4)
    s = Synth(73)
    U = s.gauge(dims).numpy()
    lat = _lat(U, ANTI, 0.12)
    X0 = _cuda(s.gaussian_spinor(dims, 2).numpy())
    with pytest.raises(cola.ColaError):
        lat.eigensolve(X0, system=cola.COLA_SYS_PROPAGATOR)
    with pytest.raises(cola.ColaError):
        lat.eigensolve(X0, tol=0.0)
    # a starting vector with nothing left once the vectors before it are projected out (here
    # a zero vector; a copy of an earlier start is not one, since that vector has moved by
    # the time the copy is reached): a breakdown status, nothing raised
    dead = torch.stack([X0[0], torch.zeros_like(X0[0])])
    lam, X, info = lat.eigensolve(dead)
    assert info["status"] == cola.COLA_BREAKDOWN


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP64, cola.COLA_CG_FP32_DEFECT])
def test_deflated_cg(scheme):
    """Deflation with the 4 lowest modes of S^H S on 4^4: the oracle-checked residual meets
    the tolerance and the solution is the oracle's deflated CG run on the GPU's
    eigenpairs; a right-hand side inside the span of the modes is solved by the deflated
    guess alone (no CG iteration)."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    s = Synth(74)
    U = s.gauge(dims, mix=0.9).numpy()
    X0 = s.gaussian_spinor(dims, 4).numpy()
    b = s.gaussian_spinor(dims, 2).numpy()
    lat = _lat(U, ANTI, kappa)
    lam, X, info = lat.eigensolve(_cuda(X0), system=cola.COLA_SYS_SCHUR, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    _, i0 = lat.cg(_cuda(b), system=cola.COLA_SYS_SCHUR, scheme=scheme, tol=1e-10)
    xd, idf = lat.cg_deflated(_cuda(b), X, lam, system=cola.COLA_SYS_SCHUR, scheme=scheme,
                              tol=1e-10)
    assert idf["status"] == cola.COLA_OK, idf
    assert idf["iterations"] <= i0["iterations"] + 1, (idf, i0)
    Xh = X.cpu().numpy()
    xs = xd.cpu().numpy()
    for q in range(2):
        be = _even(b[q])
        r = _even(apply_A(U, xs[q], kappa, ANTI, 1)) - be
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(be)
        g = eigen.deflated_guess(Xh, np.array(lam), b[q], system=1)
        xo, _ = eigen.cg_from(U, b[q], g, kappa, ANTI, system=1, tol=1e-12)
        assert rel(xs[q], xo) < 1e-7
    # b in the span of the modes: x0 = sum_i x_i <x_i, b> / lambda_i is the solution
    c = np.array([1.0, -0.5j, 0.25, 2.0 + 1.0j])
    bs = np.tensordot(c, Xh, axes=1)[None]
    xd, idf = lat.cg_deflated(_cuda(bs), X, lam, system=cola.COLA_SYS_SCHUR, scheme=scheme,
                              tol=1e-8)
    assert idf["status"] == cola.COLA_OK and idf["iterations"] == 0, idf
    want = np.tensordot(c / np.array(lam), Xh, axes=1)
    assert rel(xd.cpu().numpy()[0], want) < 1e-9
