"""Pins of the multi-shift CG oracle.

Against dense solves of (A + sigma) x = b (A = M^H M, or S^H S with S the dense Schur
complement) on a 2x2x2x4 lattice; on 4^4 every shifted solution's true residual,
recomputed by applying A, and the unshifted member against the oracle's C CG.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, multishift
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import rel

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
SHIFTS = [0.0, 0.02, 0.3, 1.7]


@pytest.mark.parametrize("system", [0, 1])
def test_multishift_matches_dense_solves(system):
    dims = (2, 2, 2, 4)
    s = Synth(5)
    U = s.gauge(dims, mix=0.6).numpy()
    b = s.gaussian_spinor(dims).numpy()[0]
    kappa = 0.11
    x, it = multishift.multishift_cg(U, b, SHIFTS, kappa, GENERIC, system=system, tol=1e-13)
    M = dense.wilson_matrix(U, kappa, GENERIC)
    if system == 0:
        A = M.conj().T @ M
        rows = np.ones(M.shape[0], dtype=bool)
    else:
        S = dense.schur_matrix(M, dims)
        A = S.conj().T @ S
        rows = dense.parity_vector(dims) == 0
    bv = dense.to_vec(b)[rows]
    for sig, xs in zip(SHIFTS, x):
        want = np.linalg.solve(A + sig * np.eye(A.shape[0]), bv)
        got = dense.to_vec(xs)
        assert rel(got[rows], want) < 1e-10, sig
        assert np.all(got[~rows] == 0)


@pytest.mark.parametrize("system", [0, 1])
def test_multishift_residuals_and_unshifted_member(system):
    dims = (4, 4, 4, 4)
    s = Synth(6)
    U = s.gauge(dims).numpy()
    b = s.gaussian_spinor(dims).numpy()[0]
    kappa, tol = 0.12, 1e-10
    x, it = multishift.multishift_cg(U, b, SHIFTS, kappa, GENERIC, system=system, tol=tol)
    be = b if system == 0 else np.where(oracle.parity_mask(dims)[..., None, None], b, 0)
    for sig, xs in zip(SHIFTS, x):
        r = be - multishift.apply_A(U, xs, kappa, GENERIC, system) - sig * xs
        assert np.linalg.norm(r) <= 2 * tol * np.linalg.norm(be), sig
    x0, n0, _ = oracle.cg(U, b, kappa, GENERIC, system=system, tol=tol)
    assert rel(x[0], x0) < 1e-7
    # the unshifted member converges last: the shared iteration count is its own
    assert abs(it - n0) <= 1
