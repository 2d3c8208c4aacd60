"""Configurations outside the small parity lattice, through the C ABI:

* extent-2 lattices (2^4 and 2x2x2x4), where the forward and backward neighbour
  of a site are the same site and both hops add: every operator, FP64 / FP32 /
  FP16, 1 and 12 right-hand sides, against the dense matrix assembled block by
  block (a third, independent route to M), and FP64 CG against a dense solve;
* the 48^3x96 clover workload with 12 right-hand sides in the library's default
  launch shapes (FP32, 8x4 tiles, links staged in LDS, clover epilogues): M on
  sampled sites, and the 12-source propagator solve with FP32 inner / FP64
  outer defect correction, its residual M x - b evaluated by the oracle at the
  origin, its eight neighbours and sampled sites of both parities;
* block CG at the 32^3x64 shape (12 point sources, FP16 inner), residuals
  checked the same way;
* the launch-shape tuner: tuned hops are bitwise the default-shape hops, and a
  tuned solve reaches the oracle-checked tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import dense
from paper_2302_00850_amd.synth import Synth, bc_phases, point_sources
from tests._util import assert_close, rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

ANTI = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
TOL = {0: 1e-13, 2: 2e-6, 3: 4e-3}


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _lat(U, bc, kappa, csw=0.0, flags=0):
    lat = cola.Lattice(tuple(U.shape[:4][::-1]), kappa, bc, csw, flags)
    lat.set_gauge(torch.from_numpy(U).cuda())
    return lat


# ------------------------------------------------------------ extent-2 lattices

SMALL = [(2, 2, 2, 2), (2, 2, 2, 4)]


def _dense_ops(U, kappa, bc, csw):
    dims = tuple(U.shape[:4][::-1])
    A = oracle.clover(U, kappa, csw) if csw else None
    M = dense.wilson_matrix(U, kappa, bc, clover=A)
    par = dense.parity_vector(dims)
    S = dense.schur_matrix(M, dims)
    return M, S, par == 0


@pytest.mark.parametrize("dims", SMALL)
@pytest.mark.parametrize("prec", [0, 2, 3])
@pytest.mark.parametrize("nrhs", [1, 12])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_extent2_operators_match_dense(dims, prec, nrhs, csw):
    kappa = 0.118 if csw else 0.12
    s = Synth(404)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims, nrhs).numpy()
    M, S, even = _dense_ops(U, kappa, GENERIC, csw)
    lat = _lat(U, GENERIC, kappa, csw)
    n = 12 * int(np.prod(dims))
    D = (np.eye(n) - M) / kappa if not csw else None  # hop matrix (plain Wilson only)
    cases = [(cola.COLA_OP_M, -1, M), (cola.COLA_OP_MDAG, -1, M.conj().T),
             (cola.COLA_OP_MDAGM, -1, M.conj().T @ M),
             (cola.COLA_OP_SCHUR, 0, S), (cola.COLA_OP_SCHUR_DAG, 0, S.conj().T),
             (cola.COLA_OP_SCHUR_DAGSCHUR, 0, S.conj().T @ S)]
    if D is not None:
        cases += [(cola.COLA_OP_HOP, 0, D), (cola.COLA_OP_HOP, 1, D),
                  (cola.COLA_OP_HOP_DAG, 0, D.conj().T)]
    for op, parity, mat in cases:
        hop = op in (cola.COLA_OP_HOP, cola.COLA_OP_HOP_DAG)
        in_par = 1 - parity if hop else parity
        pin = lat.pack(_cuda(psi), prec, in_par)
        out = lat.empty_packed(prec, nrhs, parity)
        lat.dslash(out, pin, op, parity, prec, nrhs)
        got = lat.unpack(out, prec, nrhs, parity).cpu().numpy().reshape(nrhs, n)
        src = lat.unpack(pin, prec, nrhs, in_par).cpu().numpy().reshape(nrhs, n)
        if parity < 0:
            ref = src @ mat.T
        elif hop:
            rows = even if parity == 0 else ~even
            ref = np.zeros_like(src)
            ref[:, rows] = src[:, ~rows] @ mat[np.ix_(rows, ~rows)].T
        else:
            ref = np.zeros_like(src)
            ref[:, even] = src[:, even] @ mat.T
        tol = TOL[prec] * (4 if op in (cola.COLA_OP_MDAGM, cola.COLA_OP_SCHUR_DAGSCHUR) else 1)
        assert_close(got, ref, tol, (dims, op, parity, prec, nrhs, csw))


@pytest.mark.parametrize("dims", SMALL)
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_extent2_cg_matches_dense_solve(dims, csw):
    kappa = 0.118 if csw else 0.12
    s = Synth(405)
    U = s.gauge(dims).numpy()
    b = s.gaussian_spinor(dims, 1).numpy()
    M, S, even = _dense_ops(U, kappa, ANTI, csw)
    lat = _lat(U, ANTI, kappa, csw)
    bv = b[0].reshape(-1)
    # full lattice: M^H M x = b
    x, info = lat.cg(_cuda(b), system=cola.COLA_SYS_MDAGM, scheme=cola.COLA_CG_FP64, tol=1e-12)
    assert info["status"] == cola.COLA_OK, info
    want = np.linalg.solve(M.conj().T @ M, bv)
    assert_close(x.cpu().numpy()[0].reshape(-1), want, 1e-10)
    # even sites: S^H S x_e = b_e
    x, info = lat.cg(_cuda(b), system=cola.COLA_SYS_SCHUR, scheme=cola.COLA_CG_FP64, tol=1e-12)
    assert info["status"] == cola.COLA_OK, info
    want = np.zeros_like(bv)
    want[even] = np.linalg.solve(S.conj().T @ S, bv[even])
    assert_close(x.cpu().numpy()[0].reshape(-1), want, 1e-10)
    # propagator: M x = b, every mixed scheme
    want = np.linalg.solve(M, bv)
    for scheme in (cola.COLA_CG_FP64, cola.COLA_CG_FP32_RELIABLE, cola.COLA_CG_FP32_DEFECT,
                   cola.COLA_CG_FP16_DEFECT):
        x, info = lat.cg(_cuda(b), system=cola.COLA_SYS_PROPAGATOR, scheme=scheme, tol=1e-11)
        assert info["status"] == cola.COLA_OK, (scheme, info)
        assert_close(x.cpu().numpy()[0].reshape(-1), want, 1e-9, scheme)


# --------------------------------------------------------- full-size workloads

def _coords(dims, sites):
    lx, ly, lz, lt = dims
    s = np.asarray(sites)
    return np.stack([s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)], -1)


def _index(dims, c):
    lx, ly, lz, _ = dims
    return c[..., 0] + lx * (c[..., 1] + ly * (c[..., 2] + lz * c[..., 3]))


def _check_sites(dims, n, seed):
    """The origin, its eight neighbours, and n random sites of each parity."""
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    o = np.zeros((9, 4), dtype=np.int64)
    for mu in range(4):
        o[1 + 2 * mu, mu] = 1
        o[2 + 2 * mu, mu] = dims[mu] - 1
    picks = rng.choice(V, size=8 * n, replace=False)
    par = _coords(dims, picks).sum(-1) % 2
    picks = np.concatenate([picks[par == 0][:n], picks[par == 1][:n]])
    return np.concatenate([_index(dims, o), picks, [V - 1]])


def _gather(field, sites):
    """Rows of a canonical (nrhs, Lt, Lz, Ly, Lx, 4, 3) device field at lexicographic
    sites, as a host array (nrhs, n, 4, 3)."""
    nr = field.shape[0]
    idx = torch.as_tensor(np.asarray(sites), device=field.device)
    return field.reshape(nr, -1, 4, 3).index_select(1, idx).cpu().numpy()


C5 = (48, 48, 48, 96)


def test_c5_clover_M_12rhs_default_shapes():
    """48^3x96 clover (kappa 0.118, c_sw 1), 12 rhs, FP32: M = A - kappa D on the full
    lattice runs two 12-rhs hops with the clover+xpay epilogue in the default launch
    shape (8x4 tiles, links staged in LDS); every rhs checked by the oracle on sampled
    sites, corners included."""
    kappa, csw = 0.118, 1.0
    s = Synth(21, device="cuda", rng="torch")
    U = s.gauge(C5)
    lat = cola.Lattice(C5, kappa, ANTI, csw)
    lat.set_gauge(U)
    Uh = U.cpu().numpy()
    del U
    psi = s.gaussian_spinor(C5, 12)
    pin = lat.pack(psi, cola.COLA_FP32, -1)
    del psi
    out = lat.empty_packed(cola.COLA_FP32, 12, -1)
    lat.dslash(out, pin, cola.COLA_OP_M, -1, cola.COLA_FP32, 12)
    sites = _check_sites(C5, 192, 5)
    got = _gather(lat.unpack(out, cola.COLA_FP32, 12, -1), sites)
    del out
    torch.cuda.empty_cache()
    src = lat.unpack(pin, cola.COLA_FP32, 12, -1)
    for q in range(12):
        sq = src[q].cpu().numpy()
        ref = oracle.apply_M_sites(Uh, sq, kappa, ANTI, sites, csw=csw)
        assert_close(got[q], ref, 2e-6, q)
    lat.close()


def _propagator_site_residuals(Uh, x, b, dims, kappa, csw, sites):
    """max over columns and sites of |(M x)(s) - b(s)| / |b|, by the oracle."""
    worst = 0.0
    bs = _gather(b, sites)
    nb = torch.linalg.vector_norm(b.reshape(b.shape[0], -1), dim=1).cpu().numpy()
    for q in range(x.shape[0]):
        xq = x[q].cpu().numpy()
        mx = oracle.apply_M_sites(Uh, xq, kappa, ANTI, sites, csw=csw)
        r = np.linalg.norm((mx - bs[q]).reshape(len(sites), -1), axis=1).max() / nb[q]
        worst = max(worst, float(r))
    return worst


def test_c5_propagator_fp32_defect_sampled_residual():
    """The 48^3x96 clover workload: 12 point sources, M x = b through the even-odd
    Schur normal equations, FP32 inner iterations inside FP64 defect correction to
    1e-10, default launch shapes.  The oracle evaluates M x - b at the origin, its
    eight neighbours, 2 x 192 sampled sites and the last site, for every column."""
    kappa, csw = 0.118, 1.0
    U = Synth(0, device="cuda", rng="torch").gauge(C5)
    lat = cola.Lattice(C5, kappa, ANTI, csw)
    lat.set_gauge(U)
    Uh = U.cpu().numpy()
    del U
    b = point_sources(C5, device="cuda")
    x, info = lat.cg(b, system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP32_DEFECT,
                     tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    lat.close()
    sites = _check_sites(C5, 192, 6)
    worst = _propagator_site_residuals(Uh, x, b, C5, kappa, csw, sites)
    # a site's share of |M x - b| is at most the whole, which meets the tolerance
    assert worst <= 1.1e-10, worst
    assert max(info["true_rel_residual"]) <= 1e-10, info
    # the solution is not trivially small where the residual is checked
    assert float(torch.linalg.vector_norm(x[0].reshape(-1, 12)[0])) > 0.5


def test_block_cg_c3_propagator_sampled_residual():
    """Block CG (one Krylov space for the 12 point sources) at the 32^3x64 shape with
    FP16 inner iterations and FP64 defect correction; the oracle checks M x - b on
    sampled sites of every column, and the lockstep solver reaches the same x."""
    dims = (32, 32, 32, 64)
    kappa = 0.12
    U = Synth(0, device="cuda", rng="torch").gauge(dims)
    lat = cola.Lattice(dims, kappa, ANTI)
    lat.set_gauge(U)
    Uh = U.cpu().numpy()
    del U
    b = point_sources(dims, device="cuda")
    x, info = lat.cg(b, system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP16_DEFECT,
                     tol=1e-10, block=1)
    assert info["status"] == cola.COLA_OK, info
    sites = _check_sites(dims, 192, 7)
    assert _propagator_site_residuals(Uh, x, b, dims, kappa, 0.0, sites) <= 1.1e-10
    assert max(info["true_rel_residual"]) <= 1e-10, info
    x2, info2 = lat.cg(b, system=cola.COLA_SYS_PROPAGATOR, scheme=cola.COLA_CG_FP16_DEFECT,
                       tol=1e-10, block=0)
    assert info2["status"] == cola.COLA_OK
    assert rel(x.cpu().numpy(), x2.cpu().numpy()) < 1e-7
    lat.close()


# ------------------------------------------------------------------ tuner

@pytest.mark.parametrize("prec", [cola.COLA_FP32, cola.COLA_FP16])
def test_tuner_bitwise_and_tuned_solve(prec, tmp_path):
    """With tuning on, the first use of each hop key times every candidate launch shape
    and keeps the fastest; any shape gives bitwise the default shape's output.  A solve
    with tuned shapes reaches the tolerance the oracle recomputes."""
    dims = (8, 8, 8, 16)
    kappa = 0.12
    s = Synth(31)
    U = s.gauge(dims).numpy()
    psi = s.gaussian_spinor(dims, 12).numpy()
    lat = _lat(U, ANTI, kappa)
    pin = lat.pack(_cuda(psi), prec, 1)
    ref = lat.empty_packed(prec, 12, 0)
    lat.dslash(ref, pin, cola.COLA_OP_HOP, 0, prec, 12)
    tuned = cola.Lattice(dims, kappa, ANTI)
    tuned.set_gauge(_cuda(U))
    cola.cola_set_tuning(tuned.h, 1)
    out = tuned.empty_packed(prec, 12, 0)
    tuned.dslash(out, pin, cola.COLA_OP_HOP, 0, prec, 12)
    assert "hop:" in cola.cola_tune_dump(tuned.h)
    out2 = tuned.empty_packed(prec, 12, 0)
    tuned.dslash(out2, pin, cola.COLA_OP_HOP, 0, prec, 12)  # the cached shape
    assert torch.equal(out, ref) and torch.equal(out2, ref)
    # the tuned shapes persist: written to a file, read back by a fresh handle, whose hop
    # (tuning off) then takes the stored shape -- still bitwise the default output
    path = str(tmp_path / "tune.txt")
    n = cola.cola_tune_save(tuned.h, path)
    assert n >= 1
    assert any(f"hop:{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}:p{prec}:r12" in line
               for line in open(path))
    fresh = cola.Lattice(dims, kappa, ANTI)
    fresh.set_gauge(_cuda(U))
    assert cola.cola_tune_load(fresh.h, path) == n
    out3 = fresh.empty_packed(prec, 12, 0)
    fresh.dslash(out3, pin, cola.COLA_OP_HOP, 0, prec, 12)
    assert torch.equal(out3, ref)
    fresh.close()
    b = point_sources(dims).numpy()
    scheme = cola.COLA_CG_FP32_DEFECT if prec == cola.COLA_FP32 else cola.COLA_CG_FP16_DEFECT
    x, info = tuned.cg(_cuda(b), system=cola.COLA_SYS_PROPAGATOR, scheme=scheme, tol=1e-10)
    assert info["status"] == cola.COLA_OK, info
    xs = x.cpu().numpy()
    for q in (0, 4, 11):
        assert rel(oracle.apply_M(U, xs[q], kappa, ANTI), b[q]) <= 1.1e-10
    tuned.close()
    lat.close()
