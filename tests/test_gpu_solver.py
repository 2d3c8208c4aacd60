"""GPU CG solvers and fermion force against the FP64 oracle (through the C ABI).

FP64 CG: both sides run exactly N iterations (N = the oracle's converged
count) and the iterates agree to 1e-12 relative.  Mixed and multi-RHS
schemes: the true residual of the GPU solution, recomputed by the oracle, is
at most the requested tolerance.  Force: GPU kernel fed the oracle's X and Y
agrees with the oracle force to 1e-12; the autograd path agrees to 1e-8.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources
from tests._util import assert_close, rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

ANTI = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
DIMS = (6, 4, 4, 10)
KAPPA = 0.12


@pytest.fixture(scope="module")
def fields():
    s = Synth(202)
    U = s.gauge(DIMS).numpy()
    b = s.gaussian_spinor(DIMS, 12).numpy()
    return U, b


def _lat(U, bc, csw=0.0, kappa=KAPPA):
    lat = cola.Lattice(tuple(U.shape[:4][::-1]), kappa, bc, csw)
    lat.set_gauge(torch.from_numpy(U).cuda())
    return lat


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _even(dims):
    return oracle.parity_mask(dims)[..., None, None]


def _normal_residual(U, x, b, system, kappa, bc, A=None, Ai=None):
    if system == cola.COLA_SYS_MDAGM:
        ax = oracle.apply_M(U, oracle.apply_M(U, x, kappa, bc, clover=A), kappa, bc, clover=A,
                            dagger=True)
        return rel(ax, b)
    be = np.where(_even(DIMS), b, 0)
    ax = oracle.apply_schur(U, oracle.apply_schur(U, x, kappa, bc, A, Ai), kappa, bc, A, Ai,
                            dagger=True)
    return rel(ax, be)


@pytest.mark.parametrize("system,fuse", [(cola.COLA_SYS_MDAGM, "1"), (cola.COLA_SYS_MDAGM, "0"),
                                         (cola.COLA_SYS_SCHUR, "1"), (cola.COLA_SYS_SCHUR, "0")])
def test_cg_fp64_fixed_iterations_match_oracle(fields, system, fuse, monkeypatch):
    """fuse: the even-odd CG update inside the last hop (1) or as its own kernel (0)."""
    monkeypatch.setenv("COLA_CG_FUSE", fuse)
    U, b = fields
    sysid = 0 if system == cola.COLA_SYS_MDAGM else 1
    _, n, _ = oracle.cg(U, b[0], KAPPA, GENERIC, system=sysid, tol=1e-10)
    assert n > 10
    x_ref, _, _ = oracle.cg(U, b[0], KAPPA, GENERIC, system=sysid, fixed_iters=n)
    lat = _lat(U, GENERIC)
    x, info = lat.cg(_cuda(b[:1]), system=system, scheme=cola.COLA_CG_FP64, tol=1e-300,
                     max_iter=n)
    assert info["iterations"] == n and info["status"] == cola.COLA_NOT_CONVERGED
    assert_close(x.cpu().numpy()[0], x_ref, 1e-12)


SCHEMES = [cola.COLA_CG_FP64, cola.COLA_CG_FP32_RELIABLE, cola.COLA_CG_FP16_DEFECT,
           cola.COLA_CG_FP32_DEFECT]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("system", [cola.COLA_SYS_MDAGM, cola.COLA_SYS_SCHUR])
@pytest.mark.parametrize("nrhs", [1, 12])
def test_cg_schemes_reach_tolerance(fields, scheme, system, nrhs):
    U, b = fields
    tol = 1e-10
    src = b[:nrhs] if nrhs == 1 else point_sources(DIMS).numpy()
    lat = _lat(U, ANTI)
    x, info = lat.cg(_cuda(src), system=system, scheme=scheme, tol=tol)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(nrhs):
        r = _normal_residual(U, xs[q], src[q], system, KAPPA, ANTI)
        assert r <= 1.05 * tol, (scheme, system, q, r, info)
        assert info["true_rel_residual"][q] <= tol
    if system == cola.COLA_SYS_SCHUR:
        assert np.all(np.where(_even(DIMS), 0, xs) == 0)


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP16_DEFECT, cola.COLA_CG_FP32_DEFECT])
@pytest.mark.parametrize("system", [cola.COLA_SYS_SCHUR, cola.COLA_SYS_PROPAGATOR])
def test_block_cg_reaches_tolerance(fields, scheme, system):
    """Block CG (one Krylov space for the 12 point sources) inside defect correction."""
    U, b = fields
    src = point_sources(DIMS).numpy()
    lat = _lat(U, ANTI)
    x, info = lat.cg(_cuda(src), system=system, scheme=scheme, tol=1e-10, block=1)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(12):
        if system == cola.COLA_SYS_SCHUR:
            r = _normal_residual(U, xs[q], src[q], system, KAPPA, ANTI)
            assert r <= 1.05e-10, (q, r, info)
        else:
            assert rel(oracle.apply_M(U, xs[q], KAPPA, ANTI), src[q]) <= 1.1e-10
    # lockstep twin: the same solutions (to the solver tolerance, relative to cond)
    x2, info2 = lat.cg(_cuda(src), system=system, scheme=scheme, tol=1e-10, block=0)
    assert rel(xs, x2.cpu().numpy()) < 1e-7


@pytest.mark.parametrize("nrhs", [1, 2, 3, 8, 16])
def test_block_cg_column_counts(fields, nrhs):
    """Block CG with 1 to 16 columns (the unit kernels' partial wavefronts and every Gram
    row count): each column's normal-system residual, recomputed by the oracle, meets the
    tolerance."""
    U, _ = fields
    s = Synth(303 + nrhs)
    src = s.gaussian_spinor(DIMS, nrhs).numpy()
    lat = _lat(U, ANTI)
    x, info = lat.cg(_cuda(src), system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_DEFECT,
                     tol=1e-10, block=1)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(nrhs):
        r = _normal_residual(U, xs[q], src[q], cola.COLA_SYS_SCHUR, KAPPA, ANTI)
        assert r <= 1.05e-10, (nrhs, q, r)


def test_block_cg_dependent_columns(fields):
    """Duplicate and zero columns make the block Gram matrices singular; the
    deflating small solve must still converge every column."""
    U, b = fields
    src = np.stack([b[0], b[1], b[0], np.zeros_like(b[0]), 2.0 * b[1]])
    lat = _lat(U, ANTI)
    x, info = lat.cg(_cuda(src), system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP32_DEFECT,
                     tol=1e-10, block=1)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    assert np.all(xs[3] == 0)
    for q in (0, 1, 2, 4):
        assert _normal_residual(U, xs[q], src[q], cola.COLA_SYS_SCHUR, KAPPA, ANTI) <= 1.05e-10


def test_block_cg_rejected_where_unsupported(fields):
    U, b = fields
    lat = _lat(U, ANTI)
    with pytest.raises(cola.ColaError):
        lat.cg(_cuda(b[:2]), system=cola.COLA_SYS_MDAGM, scheme=cola.COLA_CG_FP16_DEFECT, block=1)
    with pytest.raises(cola.ColaError):
        lat.cg(_cuda(b[:2]), system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, block=1)


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP64, cola.COLA_CG_FP32_DEFECT])
def test_cg_clover_schur(fields, scheme):
    U, b = fields
    kappa, csw = 0.118, 1.0
    A = oracle.clover(U, kappa, csw)
    Ai = oracle.site_inverse(A)
    lat = _lat(U, ANTI, csw=csw, kappa=kappa)
    x, info = lat.cg(_cuda(b[:2]), system=cola.COLA_SYS_SCHUR, scheme=scheme, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in range(2):
        assert _normal_residual(U, xs[q], b[q], cola.COLA_SYS_SCHUR, kappa, ANTI, A, Ai) <= 1.05e-10


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("csw", [0.0, 1.0])
@pytest.mark.parametrize("system", [cola.COLA_SYS_SCHUR, cola.COLA_SYS_MDAGM])
def test_cg_fused_update_matches_separate(fields, scheme, csw, system, monkeypatch):
    """The CG update fused into the last hop of S^dag S (even-odd) or the two parity
    hops of M^dag (full lattice) against the separate update kernel: both reach the
    tolerance, in about as many iterations, at the same solutions (to the tolerance
    times the condition number)."""
    U, b = fields
    kappa = 0.118 if csw else KAPPA
    A = oracle.clover(U, kappa, csw) if csw else None
    Ai = oracle.site_inverse(A) if csw else None
    src = point_sources(DIMS).numpy()
    lat = _lat(U, ANTI, csw=csw, kappa=kappa)
    out = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("COLA_CG_FUSE", fuse)
        x, info = lat.cg(_cuda(src), system=system, scheme=scheme, tol=1e-10)
        assert info["status"] == cola.COLA_OK, (fuse, info)
        out[fuse] = (x.cpu().numpy(), info)
    xs = out["1"][0]
    for q in range(12):
        r = _normal_residual(U, xs[q], src[q], system, kappa, ANTI, A, Ai)
        assert r <= 1.05e-10, (q, r)
    n0, n1 = out["0"][1]["iterations"], out["1"][1]["iterations"]
    assert abs(n1 - n0) <= max(2, n0 // 10), (n0, n1)
    assert rel(xs, out["0"][0]) < 1e-7


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP16_DEFECT, cola.COLA_CG_FP32_DEFECT])
@pytest.mark.parametrize("shape", ["2,16,0,1", "1,16,-1,2", "1,16,0,1,2,2,1", "2,16,5,1,2,2,1",
                                   "3,16,0,1,2,2"])
def test_cg_fused_update_launch_shapes(fields, scheme, shape, monkeypatch):
    """The fused CG update under launch shapes other than the default (several rhs per
    lane, resident and ragged grids, time chunks, tiles, staged links): the solve reaches
    the tolerance at the default shape's solutions."""
    U, b = fields
    src = point_sources(DIMS).numpy()
    lat = _lat(U, GENERIC)
    monkeypatch.delenv("COLA_HOP_SHAPE", raising=False)
    x0, _ = lat.cg(_cuda(src), system=cola.COLA_SYS_SCHUR, scheme=scheme, tol=1e-10)
    monkeypatch.setenv("COLA_HOP_SHAPE", shape)
    x, info = lat.cg(_cuda(src), system=cola.COLA_SYS_SCHUR, scheme=scheme, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in (0, 5, 11):
        assert _normal_residual(U, xs[q], src[q], cola.COLA_SYS_SCHUR, KAPPA, GENERIC) <= 1.05e-10
    assert rel(xs, x0.cpu().numpy()) < 1e-7


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_propagator_solves_M(fields, csw):
    U, b = fields
    kappa = 0.118 if csw else KAPPA
    A = oracle.clover(U, kappa, csw) if csw else None
    lat = _lat(U, GENERIC, csw=csw, kappa=kappa)
    x, info = lat.cg(_cuda(b[:1]), system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP64,
                     tol=1e-12)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()[0]
    r = rel(oracle.apply_M(U, xs, kappa, GENERIC, clover=A), b[0])
    assert r <= 1.1e-12  # the full-lattice residual meets tol
    assert r == pytest.approx(info["true_rel_residual"][0], rel=1e-3, abs=1e-14)


def test_cg_not_converged_and_warm_start(fields):
    U, b = fields
    lat = _lat(U, ANTI)
    x, info = lat.cg(_cuda(b[:1]), system=cola.COLA_SYS_SCHUR, tol=1e-10, max_iter=5)
    assert info["status"] == cola.COLA_NOT_CONVERGED and info["iterations"] == 5
    assert info["true_rel_residual"][0] > 1e-10
    # resume from the partial solution
    x2, info2 = lat.cg(_cuda(b[:1]), system=cola.COLA_SYS_SCHUR, tol=1e-10, x0=x)
    assert info2["status"] == cola.COLA_OK
    x3, info3 = lat.cg(_cuda(b[:1]), system=cola.COLA_SYS_SCHUR, tol=1e-10, x0=x2)
    assert info3["iterations"] == 0 and info3["status"] == cola.COLA_OK


def test_cg_breakdown_on_nan(fields):
    U, b = fields
    lat = _lat(U, ANTI)
    bad = b[:1].copy()
    bad[0, 0, 0, 0, 0, 0, 0] = np.nan
    _, info = lat.cg(_cuda(bad), system=cola.COLA_SYS_MDAGM, tol=1e-10)
    assert info["status"] == cola.COLA_BREAKDOWN


def test_cg_duplicate_and_zero_columns(fields):
    U, b = fields
    lat = _lat(U, ANTI)
    src = np.stack([b[0], b[0], np.zeros_like(b[0])])
    x, info = lat.cg(_cuda(src), system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP16_DEFECT,
                     tol=1e-10)
    assert info["status"] == cola.COLA_OK
    xs = x.cpu().numpy()
    assert np.array_equal(xs[0], xs[1])
    assert np.all(xs[2] == 0)


# ------------------------------------------------------------------- force

@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("bc", ["anti", "generic"])
def test_force_kernel_matches_oracle(fields, mode, bc):
    U, b = fields
    bcv = ANTI if bc == "anti" else GENERIC
    s = Synth(303)
    X = s.gaussian_spinor(DIMS)[0].numpy()
    Y = s.gaussian_spinor(DIMS)[0].numpy()
    lat = _lat(U, bcv)
    F = lat.force(_cuda(X), _cuda(Y), mode).cpu().numpy()
    ref = oracle.force(U, X, Y, KAPPA, bcv, mode=mode)
    assert_close(F, ref, 1e-13, "force", 36)


def test_pseudofermion_action_autograd(fields):
    U, b = fields
    s = Synth(404)
    eta = s.gaussian_spinor(DIMS)[0].numpy()
    phi = oracle.apply_M(U, eta, KAPPA, ANTI, dagger=True)
    lat = _lat(U, ANTI)
    Ut = torch.from_numpy(U).cuda().requires_grad_(True)
    S = cola.PseudofermionAction.apply(Ut, _cuda(phi), lat, 1e-12)
    S.backward()
    X, _, _ = oracle.cg(U, phi, KAPPA, ANTI, system=0, tol=1e-13)
    Y = oracle.apply_M(U, X, KAPPA, ANTI)
    S_ref = np.vdot(phi, X).real
    assert abs(S.item() - S_ref) <= 1e-10 * abs(S_ref)
    assert abs(S.item() - np.vdot(eta, eta).real) <= 1e-9 * abs(S_ref)
    G_ref = oracle.force(U, X, Y, KAPPA, ANTI, mode=0)
    assert rel(Ut.grad.cpu().numpy(), G_ref) <= 1e-8


@pytest.mark.parametrize("scheme", [cola.COLA_CG_FP64, cola.COLA_CG_FP32_RELIABLE,
                                    cola.COLA_CG_FP16_DEFECT, cola.COLA_CG_FP32_DEFECT])
@pytest.mark.parametrize("system", [cola.COLA_SYS_MDAGM, cola.COLA_SYS_SCHUR])
def test_captured_iteration_blocks_match_direct_launches(fields, scheme, system, monkeypatch):
    """With COLA_GRAPHS=1 small solves replay their iteration blocks as HIP graphs: three
    solves in a row (each replaying the graphs captured by the first, with the solver's own
    direct launches and host reads between the replays) give bitwise the solution and
    iteration count of the same solve launched kernel by kernel."""
    U, b = fields
    src = b[:3] if scheme != cola.COLA_CG_FP64 else b[:1]
    lat = _lat(U, ANTI)
    monkeypatch.setenv("COLA_GRAPHS", "0")
    x0, i0 = lat.cg(_cuda(src), system=system, scheme=scheme, tol=1e-10)
    assert i0["status"] == cola.COLA_OK, i0
    monkeypatch.setenv("COLA_GRAPHS", "1")
    for _ in range(3):
        x1, i1 = lat.cg(_cuda(src), system=system, scheme=scheme, tol=1e-10)
        assert i1["status"] == cola.COLA_OK and i1["iterations"] == i0["iterations"], (i0, i1)
        assert torch.equal(x1, x0)
    lat.close()
