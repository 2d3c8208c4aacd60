"""The non-allocating operator entry point, through the C ABI.

cola_dslash_apply_noalloc keeps the intermediate vectors of the composed
operators in a fixed per-device workspace instead of memory the library
allocates.  Its outputs must be bitwise those of cola_dslash_apply (same
kernels, same launch shapes), over two calls in a row where the second has a
smaller input (another lattice and fewer right-hand sides, reusing the same
workspace), for every operator and precision; operators needing more than
the workspace are refused before any buffer is touched.
"""
import numpy as np
import pytest
import torch

from paper_2302_00850_amd.synth import Synth, bc_phases

pytestmark = pytest.mark.gpu

cola = pytest.importorskip("paper_2302_00850_amd.cola")

GENERIC = bc_phases((0.3, -0.5, 0.7, np.pi))
OPS = [cola.COLA_OP_HOP, cola.COLA_OP_HOP_DAG, cola.COLA_OP_M, cola.COLA_OP_MDAG,
       cola.COLA_OP_MDAGM, cola.COLA_OP_SCHUR, cola.COLA_OP_SCHUR_DAG,
       cola.COLA_OP_SCHUR_DAGSCHUR]
FULL = (cola.COLA_OP_M, cola.COLA_OP_MDAG, cola.COLA_OP_MDAGM)


def _run(dims, nrhs, prec, csw, seed):
    s = Synth(seed)
    U = s.gauge(dims)
    psi = s.gaussian_spinor(dims, nrhs).cuda()
    lat = cola.Lattice(dims, 0.118 if csw else 0.12, GENERIC, csw)
    lat.set_gauge(U.cuda())
    stream = torch.cuda.current_stream().cuda_stream
    for op in OPS:
        par = -1 if op in FULL else (1 if op in (cola.COLA_OP_HOP, cola.COLA_OP_HOP_DAG) else 0)
        out_par = -1 if op in FULL else 0
        pin = lat.pack(psi, prec, par)
        ref = lat.empty_packed(prec, nrhs, out_par)
        got = torch.full_like(ref, 0x5A)  # stale bytes must not leak into the result
        cola.cola_dslash_apply(lat.h, ref.data_ptr(), pin.data_ptr(), op, 0, prec, nrhs, stream)
        cola.cola_dslash_apply_noalloc(lat.h, got.data_ptr(), pin.data_ptr(), op, 0, prec, nrhs,
                                       stream)
        # the results at every lattice site (the packed layout pads each parity block to a
        # multiple of 64 sites, which neither entry point writes)
        a = lat.unpack(got, prec, nrhs, out_par)
        b = lat.unpack(ref, prec, nrhs, out_par)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (dims, nrhs, prec, csw, op)
        assert torch.count_nonzero(b) > 0
    lat.close()


@pytest.mark.parametrize("prec", [cola.COLA_FP64, cola.COLA_FP32, cola.COLA_FP16])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_noalloc_matches_allocating_entry_point(prec, csw):
    # first call: 8x8x8x16, 12 rhs (SdagS needs 2 x 4.7 MB of workspace in FP32);
    # second call: a smaller input on the same workspace, 6x4x4x10 with 3 rhs
    _run((8, 8, 8, 16), 12, prec, csw, 61)
    _run((6, 4, 4, 10), 3, prec, csw, 62)


def test_noalloc_refuses_oversized_workspace():
    # 32^3 x 64, FP64, 1 rhs: S needs one 201 MB odd block, above the 128 MiB workspace;
    # the call fails before any buffer is read (no gauge field is even set)
    dims = (32, 32, 32, 64)
    lat = cola.Lattice(dims, 0.12, GENERIC)
    need = cola.cola_field_bytes(lat.h, cola.COLA_FP64, 1, 0)
    assert need > (128 << 20)
    buf = torch.empty(16, dtype=torch.uint8, device="cuda")
    buf2 = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(cola.ColaError) as e:
        cola.cola_dslash_apply_noalloc(lat.h, buf.data_ptr(), buf2.data_ptr(),
                                       cola.COLA_OP_SCHUR, 0, cola.COLA_FP64, 1, None)
    assert e.value.code == cola.COLA_EINVAL and "scratch" in str(e.value)
    # the hop itself needs no workspace: without a gauge field it reports the state error
    with pytest.raises(cola.ColaError) as e:
        cola.cola_dslash_apply_noalloc(lat.h, buf.data_ptr(), buf2.data_ptr(),
                                       cola.COLA_OP_HOP, 0, cola.COLA_FP64, 1, None)
    assert e.value.code == cola.COLA_ESTATE
    lat.close()
