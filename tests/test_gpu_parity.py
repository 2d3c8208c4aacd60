"""GPU <-> FP64 oracle parity through the C ABI.

Lattices span several thread blocks with a ragged tail (Vh not a multiple of
the block size), both parities, both operator signs, real and complex
boundary phases, 1 and 12 right-hand sides.  Tolerances (relative, norm-wise):
  FP64 (18 or 12 real links)  1e-13  (rounding order only)
  FP32                        2e-6   (about 10 x single-precision epsilon)
  FP16 storage                4e-3   (inputs rounded to 11-bit mantissas)
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_00850_amd.synth import Synth, bc_phases
from tests._util import assert_close, rel

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

ANTI = bc_phases((0, 0, 0, np.pi))
GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
TOL = {0: 1e-13, 1: 1e-13, 2: 2e-6, 3: 4e-3}
DIMS = (6, 4, 4, 10)   # Vh = 480: two blocks of 256 sites, ragged tail
KAPPA = 0.12


@pytest.fixture(scope="module")
def fields():
    s = Synth(101)
    U = s.gauge(DIMS).numpy()
    psi = s.gaussian_spinor(DIMS, 12).numpy()
    return U, psi


def _lat(U, bc, csw=0.0, kappa=KAPPA, flags=0):
    lat = cola.Lattice(tuple(U.shape[:4][::-1]), kappa, bc, csw, flags)
    lat.set_gauge(torch.from_numpy(U).cuda())
    return lat


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _even(dims):
    return oracle.parity_mask(dims)[..., None, None]


@pytest.mark.parametrize("prec", [0, 2, 3])
@pytest.mark.parametrize("parity", [-1, 0, 1])
def test_pack_roundtrip(fields, prec, parity):
    U, psi = fields
    lat = _lat(U, ANTI)
    x = _cuda(psi[:3])
    packed = lat.pack(x, prec, parity)
    back = lat.unpack(packed, prec, 3, parity).cpu().numpy()
    if parity >= 0:
        m = _even(DIMS) if parity == 0 else ~_even(DIMS)
        back = np.where(m, back, 0)
        ref = np.where(m, psi[:3], 0)
    else:
        ref = psi[:3]
    tol = {0: 0, 2: 1e-7, 3: 1e-3}[prec]
    assert rel(back, ref) <= tol


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("bc", ["anti", "generic"])
@pytest.mark.parametrize("nrhs", [1, 12])
def test_hop_matches_oracle(fields, prec, parity, dagger, bc, nrhs):
    U, psi = fields
    bcv = ANTI if bc == "anti" else GENERIC
    lat = _lat(U, bcv)
    src = psi[:nrhs]
    # input lives on parity 1 - parity
    m_in = ~_even(DIMS) if parity == 0 else _even(DIMS)
    src = np.where(m_in, src, 0)
    packed_in = lat.pack(_cuda(src), prec, 1 - parity)
    out = lat.empty_packed(prec, nrhs, parity)
    lat.dslash(out, packed_in, cola.COLA_OP_HOP_DAG if dagger else cola.COLA_OP_HOP, parity,
               prec, nrhs)
    got = lat.unpack(out, prec, nrhs, parity).cpu().numpy()
    # reference on what the GPU actually read (FP16/FP32 rounding of the input)
    src_r = lat.unpack(packed_in, prec, nrhs, 1 - parity).cpu().numpy()
    ref = oracle.hop(U, np.where(m_in, src_r, 0), bcv, dagger=bool(dagger))
    m_out = _even(DIMS) if parity == 0 else ~_even(DIMS)
    ref = np.where(m_out, ref, 0)
    got = np.where(m_out, got, 0)
    assert_close(got, ref, TOL[prec], (prec, parity, dagger, bc, nrhs))


OPS = [(cola.COLA_OP_M, "M"), (cola.COLA_OP_MDAG, "Mdag"), (cola.COLA_OP_MDAGM, "MdagM"),
       (cola.COLA_OP_SCHUR, "S"), (cola.COLA_OP_SCHUR_DAG, "Sdag"),
       (cola.COLA_OP_SCHUR_DAGSCHUR, "SdagS")]


def _oracle_op(name, U, x, bc, kappa, A=None, Ai=None):
    if name == "M":
        return oracle.apply_M(U, x, kappa, bc, clover=A)
    if name == "Mdag":
        return oracle.apply_M(U, x, kappa, bc, clover=A, dagger=True)
    if name == "MdagM":
        return oracle.apply_M(U, oracle.apply_M(U, x, kappa, bc, clover=A), kappa, bc, clover=A,
                              dagger=True)
    if name == "S":
        return oracle.apply_schur(U, x, kappa, bc, A, Ai)
    if name == "Sdag":
        return oracle.apply_schur(U, x, kappa, bc, A, Ai, dagger=True)
    return oracle.apply_schur(U, oracle.apply_schur(U, x, kappa, bc, A, Ai), kappa, bc, A, Ai,
                              dagger=True)


@pytest.mark.parametrize("op,name", OPS)
@pytest.mark.parametrize("prec", [0, 2, 3])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_operators_match_oracle(fields, op, name, prec, csw):
    U, psi = fields
    kappa = 0.118 if csw else KAPPA
    lat = _lat(U, GENERIC, csw=csw, kappa=kappa)
    A = oracle.clover(U, kappa, csw) if csw else None
    Ai = oracle.site_inverse(A) if csw else None
    nrhs = 2
    schur = name.startswith("S")
    parity = 0 if schur else -1
    src = psi[:nrhs]
    if schur:
        src = np.where(_even(DIMS), src, 0)
    pin = lat.pack(_cuda(src), prec, parity)
    out = lat.empty_packed(prec, nrhs, parity)
    lat.dslash(out, pin, op, parity, prec, nrhs)
    got = lat.unpack(out, prec, nrhs, parity).cpu().numpy()
    src_r = lat.unpack(pin, prec, nrhs, parity).cpu().numpy()
    ref = np.stack([_oracle_op(name, U, s, GENERIC, kappa, A, Ai) for s in src_r])
    if schur:
        got = np.where(_even(DIMS), got, 0)
    tol = TOL[prec] * (4 if name in ("MdagM", "SdagS") else 1)
    assert_close(got, ref, tol, (name, prec, csw))


def test_compressed_links_refused_for_non_su3(fields):
    U, psi = fields
    Ub = U.copy()
    Ub[0, 0, 0, 0, 0] *= 1.001  # no longer unitary
    lat = _lat(Ub, ANTI)
    assert not lat.gauge_is_su3
    pin = lat.pack(_cuda(psi[:1]), 2, 1)
    out = lat.empty_packed(2, 1, 0)
    with pytest.raises(cola.ColaError):
        lat.dslash(out, pin, cola.COLA_OP_HOP, 0, 2, 1)
    # FP64 with all 18 reals still works and matches the oracle
    pin = lat.pack(_cuda(psi[:1]), 0, 1)
    out = lat.empty_packed(0, 1, 0)
    lat.dslash(out, pin, cola.COLA_OP_HOP, 0, 0, 1)
    got = lat.unpack(out, 0, 1, 0).cpu().numpy()[0]
    src = np.where(~_even(DIMS), psi[0], 0)
    ref = np.where(_even(DIMS), oracle.hop(Ub, src, ANTI), 0)
    assert_close(np.where(_even(DIMS), got, 0), ref, 1e-13)


def test_dslash_argument_errors(fields):
    U, psi = fields
    lat = _lat(U, ANTI)
    buf = lat.empty_packed(0, 1, 0)
    with pytest.raises(cola.ColaError):
        lat.dslash(buf, buf, cola.COLA_OP_HOP, 0, 0, 1)       # aliasing
    other = lat.empty_packed(0, 1, 1)
    with pytest.raises(cola.ColaError):
        lat.dslash(buf, other, cola.COLA_OP_HOP, 2, 0, 1)      # bad parity
    with pytest.raises(cola.ColaError):
        lat.dslash(buf, other, 99, 0, 0, 1)                    # bad op
    with pytest.raises(cola.ColaError):
        lat.dslash(buf, other, cola.COLA_OP_HOP, 0, 0, 17)     # too many rhs


SHAPES = ["1,16,0,2", "1,16,0,5", "1,64,0,10", "1,16,0,1,2,2", "1,8,0,1,4,2", "1,32,3,1,4,4",
          "2,16,0,2", "4,8,0,1,2,4", "1,16,-1,2", "3,16,0,1,2,2"]


@pytest.mark.parametrize("prec", [0, 2, 3])
def test_hop_identical_across_launch_shapes(fields, prec, monkeypatch):
    """Traversal order (time chunks, spatial tiles, XCD block order), rhs per lane and
    grid size change only which lane computes a site: outputs are bitwise identical."""
    U, psi = fields
    nrhs = 4
    lat = _lat(U, ANTI)
    pin = lat.pack(_cuda(psi[:nrhs]), prec, 1)
    ref = lat.empty_packed(prec, nrhs, 0)
    monkeypatch.delenv("COLA_HOP_SHAPE", raising=False)
    lat.dslash(ref, pin, cola.COLA_OP_HOP, 0, prec, nrhs)
    for shape in SHAPES:
        if prec == 0 and not shape.startswith("1,"):
            continue  # FP64 keeps one rhs per lane
        monkeypatch.setenv("COLA_HOP_SHAPE", shape)
        out = lat.empty_packed(prec, nrhs, 0)
        lat.dslash(out, pin, cola.COLA_OP_HOP, 0, prec, nrhs)
        assert torch.equal(out, ref), shape
    # and the fused-norm path agrees across shapes to rounding order
    monkeypatch.setenv("COLA_HOP_SHAPE", "1,16,0,1,2,2")
    a = lat.pack(_cuda(psi[:nrhs]), prec, 0)
    out = lat.empty_packed(prec, nrhs, 0)
    lat.dslash(out, a, cola.COLA_OP_SCHUR, 0, prec, nrhs)
    monkeypatch.delenv("COLA_HOP_SHAPE")
    out2 = lat.empty_packed(prec, nrhs, 0)
    lat.dslash(out2, a, cola.COLA_OP_SCHUR, 0, prec, nrhs)
    assert torch.equal(out, out2)


STAGED = ["1,16,0,1,0,0,1", "1,16,0,1,2,2,1", "1,8,7,1,0,0,1", "1,16,3,2,0,0,1",
          "1,16,0,5,0,0,1", "1,32,0,1,2,4,1", "1,16,-1,1,2,2,1", "2,32,0,1,0,0,1",
          "2,16,5,1,2,2,1", "2,32,0,2,0,0,1",
          # tiles walked in time chunks (FP32: neighbours carried in registers)
          "1,16,0,2,2,2,1", "1,16,0,5,2,4,1", "1,16,3,2,2,2,1", "1,8,-1,10,4,4,1",
          "2,16,0,5,2,2,1"]


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("op", ["hop", "schur", "clover_schur"])
def test_staged_links_identical(fields, prec, op, monkeypatch):
    """With 12 rhs the lanes of a site can stage its links in LDS; the result is bitwise
    the one of per-lane link loads, for several block sizes, grid-stride loops with a
    ragged last pass, time chunks and tiles, tiles walked in time chunks (the FP32 time
    walk with neighbours in registers), and with the fused norm and clover epilogues of
    the Schur operator."""
    U, psi = fields
    nrhs = 12
    clover = op == "clover_schur"
    lat = _lat(U, GENERIC, csw=1.0 if clover else 0.0, kappa=0.118 if clover else KAPPA)
    code = cola.COLA_OP_HOP if op == "hop" else cola.COLA_OP_SCHUR
    pin = lat.pack(_cuda(psi), prec, 1 if op == "hop" else 0)
    monkeypatch.setenv("COLA_HOP_SHAPE", "1,16,0,1,0,0,0")
    ref = lat.empty_packed(prec, nrhs, 0)
    lat.dslash(ref, pin, code, 0, prec, nrhs)
    for shape in STAGED:
        monkeypatch.setenv("COLA_HOP_SHAPE", shape)
        out = lat.empty_packed(prec, nrhs, 0)
        lat.dslash(out, pin, code, 0, prec, nrhs)
        assert torch.equal(out, ref), shape
    # and it is the oracle's hop
    if op == "hop":
        got = lat.unpack(ref, prec, nrhs, 0).cpu().numpy()
        src = np.where(~_even(DIMS), lat.unpack(pin, prec, nrhs, 1).cpu().numpy(), 0)
        want = np.where(_even(DIMS), oracle.hop(U, src, GENERIC), 0)
        assert_close(np.where(_even(DIMS), got, 0), want, TOL[prec])


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("nrhs", [5, 8, 16])
def test_hop_rhs_counts(fields, prec, nrhs):
    """Right-hand-side counts with partial wavefronts (5), the smallest staged count (8)
    and the largest (16), against the oracle."""
    U, psi0 = fields
    s = Synth(202)
    psi = s.gaussian_spinor(DIMS, nrhs).numpy()
    lat = _lat(U, GENERIC)
    src = np.where(~_even(DIMS), psi, 0)
    pin = lat.pack(_cuda(src), prec, 1)
    out = lat.empty_packed(prec, nrhs, 0)
    lat.dslash(out, pin, cola.COLA_OP_HOP, 0, prec, nrhs)
    got = np.where(_even(DIMS), lat.unpack(out, prec, nrhs, 0).cpu().numpy(), 0)
    src_r = np.where(~_even(DIMS), lat.unpack(pin, prec, nrhs, 1).cpu().numpy(), 0)
    want = np.where(_even(DIMS), oracle.hop(U, src_r, GENERIC), 0)
    assert_close(got, want, TOL[prec])


def test_hop_deterministic_and_timing_stats(fields):
    U, psi = fields
    lat = _lat(U, ANTI, flags=cola.COLA_FLAG_TIMING)
    pin = lat.pack(_cuda(psi), 3, 1)
    o1 = lat.empty_packed(3, 12, 0)
    o2 = lat.empty_packed(3, 12, 0)
    lat.dslash(o1, pin, cola.COLA_OP_HOP, 0, 3, 12)
    lat.dslash(o2, pin, cola.COLA_OP_HOP, 0, 3, 12)
    assert torch.equal(o1, o2)
    st = lat.stats()
    assert st["hop_launches"] == 2 and st["hop_seconds"] > 0
    # 8 FP16 links of 24 B + 12 rhs x (52 B in + 52 B out) per even site
    assert st["hop_bytes"] == pytest.approx(2 * 480 * (8 * 24 + 12 * 104))
