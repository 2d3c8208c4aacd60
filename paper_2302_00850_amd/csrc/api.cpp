// The C ABI (include/cola.h): argument validation, handle lifecycle, gauge
// ingest and dispatch to the operator, solver and force code.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "handle.h"

namespace cola {
int cg_solve_impl(cola_handle_t *h, void *x, const void *b, int nrhs, const cola_cg_params_t *p,
                  cola_cg_result_t *r, hipStream_t st);
int cg_multishift_impl(cola_handle_t *h, void *x, const void *b, int nshift, const double *sigma,
                       const cola_cg_params_t *p, cola_cg_result_t *r, hipStream_t st);
}

using namespace cola;

namespace {

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

bool valid_prec(int p) { return p >= COLA_FP64 && p <= COLA_FP16; }

int check_rhs(cola_handle_t *h, int nrhs) {
    if (nrhs < 1 || nrhs > kMaxRhs)
        return set_error(h, COLA_EINVAL, "nrhs must be in 1.." + std::to_string(kMaxRhs));
    // element offsets are 32-bit inside the kernels and one buffer descriptor spans
    // one component array of a block (S * nrhs elements of at most 16 bytes)
    if ((double)h->g.S * nrhs * 12.0 >= 4294967296.0 ||
        (double)h->g.S * nrhs * 16.0 >= 2147483648.0)
        return set_error(h, COLA_EINVAL, "lattice x nrhs too large for 32-bit offsets");
    return COLA_OK;
}

void free_all(cola_handle_t *h) {
    for (auto &g : h->gauge)
        if (g) hipFree(g), g = nullptr;
    for (auto &g : h->fat)
        if (g) hipFree(g), g = nullptr;
    for (void **p : {&h->clov64, &h->clovinv64, &h->clov32, &h->clovinv32})
        if (*p) hipFree(*p), *p = nullptr;
    for (auto &kv : h->cache.bufs) hipFree(kv.second.first);
    h->cache.bufs.clear();
    if (h->partial) hipFree(h->partial);
    if (h->counter) hipFree(h->counter);
    if (h->scal) hipFree(h->scal);
    if (h->active) hipFree(h->active);
    if (h->host_scal) hipHostFree(h->host_scal);
    if (h->host_active) hipHostFree(h->host_active);
    for (auto &pr : h->pending) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    for (auto e : h->event_pool) hipEventDestroy(e);
    graphs_clear(h);
    if (h->gevent) hipEventDestroy(h->gevent), h->gevent = nullptr;
    if (h->gstream) hipStreamDestroy(h->gstream), h->gstream = nullptr;
}

}  // namespace

extern "C" {

int cola_abi_version(void) { return COLA_ABI_VERSION; }

int cola_create(cola_handle_t **hp, const int dims[4], double kappa, const double bc_phase[8],
                double csw, unsigned flags) {
    if (!hp || !dims || !bc_phase) return COLA_EINVAL;
    *hp = nullptr;
    for (int mu = 0; mu < 4; ++mu)
        if (dims[mu] < 2 || dims[mu] % 2 != 0) return COLA_EINVAL;
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return COLA_EINVAL;
    const double V = (double)dims[0] * dims[1] * dims[2] * dims[3];
    if (V * 4 >= 2147483648.0) return COLA_EINVAL;
    cola_handle_t *h = new (std::nothrow) cola_handle_t;
    if (!h) return COLA_ENOMEM;
    for (int mu = 0; mu < 4; ++mu) h->dims[mu] = dims[mu];
    Geom &g = h->g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = dims[mu];
    g.Lxh = dims[0] / 2;
    g.Vh = (int)(V / 2);
    g.S = packed_stride(g.Vh);
    g.s1 = g.Lxh;
    g.s2 = g.Lxh * dims[1];
    g.s3 = g.Lxh * dims[1] * dims[2];
    g.div_xh = make_fastdiv((uint32_t)g.Lxh);
    g.div_y = make_fastdiv((uint32_t)dims[1]);
    g.div_z = make_fastdiv((uint32_t)dims[2]);
    h->kappa = kappa;
    h->csw = csw;
    h->flags = flags;
    for (int mu = 0; mu < 4; ++mu) h->phase[mu] = {bc_phase[2 * mu], bc_phase[2 * mu + 1]};
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, h->device);
        if (e == hipSuccess) {
            h->arch = prop.gcnArchName;
            const size_t colon = h->arch.find(':');  // drop feature flags
            if (colon != std::string::npos) h->arch.resize(colon);
        }
    }
    if (e == hipSuccess) e = hipMalloc(&h->partial, sizeof(double) * kRedPartialDoubles);
    if (e == hipSuccess) e = hipMalloc(&h->counter, sizeof(unsigned) * kRedCounters);
    if (e == hipSuccess) e = hipMemset(h->counter, 0, sizeof(unsigned) * kRedCounters);
    if (e == hipSuccess) e = hipMalloc(&h->scal, sizeof(double) * kScalSlots * kMaxRhs);
    if (e == hipSuccess) e = hipMemset(h->scal, 0, sizeof(double) * kScalSlots * kMaxRhs);
    if (e == hipSuccess) e = hipMalloc(&h->active, sizeof(int) * kMaxRhs);
    if (e == hipSuccess) e = hipHostMalloc(&h->host_scal, sizeof(double) * kScalSlots * kMaxRhs);
    if (e == hipSuccess) e = hipHostMalloc(&h->host_active, sizeof(int) * kMaxRhs);
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return e == hipErrorOutOfMemory ? COLA_ENOMEM : COLA_EHIP;
    }
    // the fixed workspace of cola_dslash_apply_noalloc: its address on this device
    if (scratch_address(h, &h->scratch) != COLA_OK) {
        free_all(h);
        delete h;
        return COLA_EHIP;
    }
    const char *tune = getenv("COLA_TUNE");
    if (tune) h->tune_mode = atoi(tune);
    *hp = h;
    return COLA_OK;
}

int cola_destroy(cola_handle_t *h) {
    if (!h) return COLA_EINVAL;
    hipDeviceSynchronize();
    free_all(h);
    delete h;
    return COLA_OK;
}

const char *cola_last_error(const cola_handle_t *h) { return h ? h->err.c_str() : "null handle"; }

// Pack a canonical field into the four link formats of dst (allocated on first use);
// *dev receives the largest SU(3) deviation of its links.
int pack_links(cola_handle_t *h, const void *U, void *dst[4], double *dev_out, hipStream_t st) {
    const Geom &g = h->g;
    for (int f = 0; f < 4; ++f) {
        const size_t bytes =
            (size_t)2 * 4 * link_chunks((LinkFmt)f) * link_chunk_bytes((LinkFmt)f) * g.S;
        if (!dst[f]) {
            COLA_HIP(h, hipMalloc(&dst[f], bytes));
            COLA_HIP(h, hipMemset(dst[f], 0, bytes));
        }
    }
    unsigned long long *dev;
    void *tmp;
    COLA_TRY(get_vec(h, "su3_dev", 64, &tmp));
    dev = (unsigned long long *)tmp;
    COLA_HIP(h, hipMemsetAsync(dev, 0, 8, st));
    COLA_HIP(h, launch_pack_gauge(g, U, dst[0], dst[1], dst[2], dst[3], dev, st));
    unsigned long long bits = 0;
    COLA_HIP(h, hipMemcpyAsync(&bits, dev, 8, hipMemcpyDeviceToHost, st));
    COLA_HIP(h, hipStreamSynchronize(st));
    memcpy(dev_out, &bits, 8);
    return COLA_OK;
}

// The clover blocks A = 1 - kappa csw sum sigma F[W] and A^-1 from the canonical field W.
int build_clover(cola_handle_t *h, const void *W, hipStream_t st) {
    const Geom &g = h->g;
    const size_t cb = (size_t)2 * 36 * g.S;
    for (void **p : {&h->clov64, &h->clovinv64}) {
        if (!*p) COLA_HIP(h, hipMalloc(p, cb * 16));
    }
    for (void **p : {&h->clov32, &h->clovinv32}) {
        if (!*p) COLA_HIP(h, hipMalloc(p, cb * 8));
    }
    void *badp;
    COLA_TRY(get_vec(h, "clover_bad", 64, &badp));
    COLA_HIP(h, hipMemsetAsync(badp, 0, 4, st));
    COLA_HIP(h, launch_clover_build(g, W, h->kappa, h->csw, h->clov64, h->clovinv64, h->clov32,
                                    h->clovinv32, (int *)badp, st));
    int bad = 0;
    COLA_HIP(h, hipMemcpyAsync(&bad, badp, 4, hipMemcpyDeviceToHost, st));
    COLA_HIP(h, hipStreamSynchronize(st));
    if (bad)
        return set_error(h, COLA_EINVAL,
                         std::to_string(bad) + " clover blocks are not positive definite");
    return COLA_OK;
}

int cola_set_gauge(cola_handle_t *h, const void *U, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!U) return set_error(h, COLA_EINVAL, "null gauge pointer");
    hipStream_t st = as_stream(stream);
    double d;
    h->flic = false;
    COLA_TRY(pack_links(h, U, h->gauge, &d, st));
    h->su3_dev = d;
    h->su3 = d <= 1e-12;
    if (h->csw != 0.0) {
        const int rc = build_clover(h, U, st);
        if (rc != COLA_OK) {
            h->gauge_set = false;
            return rc;
        }
    }
    h->gauge_set = true;
    return COLA_OK;
}

int cola_set_fat_gauge(cola_handle_t *h, const void *F, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!F) return set_error(h, COLA_EINVAL, "null fat-link pointer");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "set the thin links first");
    hipStream_t st = as_stream(stream);
    double d;
    h->flic = false;
    COLA_TRY(pack_links(h, F, h->fat, &d, st));
    if (!(d <= 1e-12))
        return set_error(h, COLA_EINVAL, "smeared links are not SU(3) (deviation " +
                                             std::to_string(d) + ")");
    if (h->csw != 0.0) {
        const int rc = build_clover(h, F, st);
        if (rc != COLA_OK) {
            h->gauge_set = false;
            return rc;
        }
    }
    h->flic = true;
    return COLA_OK;
}

int cola_ape_smear(cola_handle_t *h, void *F, const void *U, double alpha, int nsweeps,
                   void *stream) {
    if (!h) return COLA_EINVAL;
    if (!F || !U) return set_error(h, COLA_EINVAL, "null pointer");
    if (!std::isfinite(alpha) || nsweeps < 0)
        return set_error(h, COLA_EINVAL, "need a finite alpha and nsweeps >= 0");
    hipStream_t st = as_stream(stream);
    const size_t bytes = (size_t)h->g.Vh * 2 * 4 * 9 * 16;
    if (nsweeps == 0) {
        if (F != U) COLA_HIP(h, hipMemcpyAsync(F, U, bytes, hipMemcpyDeviceToDevice, st));
        return COLA_OK;
    }
    void *tmp;
    COLA_TRY(get_vec(h, "ape_tmp", bytes, &tmp));
    // sweeps alternate between F and the work field so that the last lands in F; a sweep
    // never reads the field it writes
    const void *src = U;
    for (int k = 0; k < nsweeps; ++k) {
        void *dst = ((nsweeps - 1 - k) % 2 == 0) ? F : tmp;
        if (dst == src) dst = dst == F ? tmp : F;  // F aliasing U on the first sweep
        COLA_HIP(h, launch_ape_sweep(h->g, src, dst, alpha, st));
        src = dst;
    }
    if (src != F) COLA_HIP(h, hipMemcpyAsync(F, src, bytes, hipMemcpyDeviceToDevice, st));
    return COLA_OK;
}

int cola_gauge_is_su3(const cola_handle_t *h) { return h && h->gauge_set && h->su3 ? 1 : 0; }

size_t cola_field_bytes(const cola_handle_t *h, int prec, int nrhs, int parity) {
    if (!h || !valid_prec(prec) || nrhs < 1 || nrhs > kMaxRhs || parity < -1 || parity > 1)
        return 0;
    const size_t b = spinor_block_bytes(h->g, spinor_fmt(prec), nrhs);
    return parity < 0 ? 2 * b : b;
}

int cola_pack_spinor(cola_handle_t *h, void *dst, const void *src, int prec, int nrhs, int parity,
                     void *stream) {
    if (!h) return COLA_EINVAL;
    if (!dst || !src) return set_error(h, COLA_EINVAL, "null pointer");
    if (!valid_prec(prec)) return set_error(h, COLA_EINVAL, "unknown precision");
    if (parity < -1 || parity > 1) return set_error(h, COLA_EINVAL, "parity must be -1, 0 or 1");
    COLA_TRY(check_rhs(h, nrhs));
    hipStream_t st = as_stream(stream);
    // clear the whole destination so padding sites are zero
    COLA_HIP(h, hipMemsetAsync(dst, 0, cola_field_bytes(h, prec, nrhs, parity), st));
    COLA_HIP(h, launch_pack_spinor(h->g, spinor_fmt(prec), dst, src, nrhs, parity, st));
    return COLA_OK;
}

int cola_unpack_spinor(cola_handle_t *h, void *dst, const void *src, int prec, int nrhs,
                       int parity, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!dst || !src) return set_error(h, COLA_EINVAL, "null pointer");
    if (!valid_prec(prec)) return set_error(h, COLA_EINVAL, "unknown precision");
    if (parity < -1 || parity > 1) return set_error(h, COLA_EINVAL, "parity must be -1, 0 or 1");
    COLA_TRY(check_rhs(h, nrhs));
    COLA_HIP(h, launch_unpack_spinor(h->g, spinor_fmt(prec), dst, src, nrhs, parity,
                                     as_stream(stream)));
    return COLA_OK;
}

int cola_dslash_apply(cola_handle_t *h, void *out, const void *in, int op, int parity, int prec,
                      int nrhs, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!out || !in) return set_error(h, COLA_EINVAL, "null pointer");
    if (out == in) return set_error(h, COLA_EINVAL, "out and in must not overlap");
    if (!valid_prec(prec)) return set_error(h, COLA_EINVAL, "unknown precision");
    if (op < COLA_OP_HOP || op > COLA_OP_SCHUR_DAGSCHUR)
        return set_error(h, COLA_EINVAL, "unknown operator");
    if ((op == COLA_OP_HOP || op == COLA_OP_HOP_DAG) && (parity < 0 || parity > 1))
        return set_error(h, COLA_EINVAL, "HOP needs the output parity 0 or 1");
    COLA_TRY(check_rhs(h, nrhs));
    return apply_op(h, out, in, op, parity, prec, nrhs, as_stream(stream));
}

int cola_dslash_apply_noalloc(cola_handle_t *h, void *out, const void *in, int op, int parity,
                              int prec, int nrhs, void *stream) {
    static_assert(kScratchBytes == COLA_NOALLOC_SCRATCH_BYTES, "workspace size in the header");
    if (!h) return COLA_EINVAL;
    if (!out || !in) return set_error(h, COLA_EINVAL, "null pointer");
    if (out == in) return set_error(h, COLA_EINVAL, "out and in must not overlap");
    if (!valid_prec(prec)) return set_error(h, COLA_EINVAL, "unknown precision");
    if (op < COLA_OP_HOP || op > COLA_OP_SCHUR_DAGSCHUR)
        return set_error(h, COLA_EINVAL, "unknown operator");
    if ((op == COLA_OP_HOP || op == COLA_OP_HOP_DAG) && (parity < 0 || parity > 1))
        return set_error(h, COLA_EINVAL, "HOP needs the output parity 0 or 1");
    COLA_TRY(check_rhs(h, nrhs));
    const size_t need = op_workspace_bytes(h, op, prec, nrhs);
    if (need > kScratchBytes)
        return set_error(h, COLA_EINVAL,
                         "operator needs " + std::to_string(need) +
                             " bytes of workspace, above the fixed " +
                             std::to_string(kScratchBytes) +
                             "-byte scratch of cola_dslash_apply_noalloc");
    if (!h->scratch) return set_error(h, COLA_ESTATE, "no workspace address for this device");
    return apply_op(h, out, in, op, parity, prec, nrhs, as_stream(stream), nullptr,
                    (char *)h->scratch);
}

int cola_cg_solve(cola_handle_t *h, void *x, const void *b, int nrhs, const cola_cg_params_t *p,
                  cola_cg_result_t *r, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!x || !b || !p) return set_error(h, COLA_EINVAL, "null pointer");
    if (x == b) return set_error(h, COLA_EINVAL, "x and b must not overlap");
    COLA_TRY(check_rhs(h, nrhs));
    if (p->system < COLA_SYS_MDAGM || p->system > COLA_SYS_PROPAGATOR)
        return set_error(h, COLA_EINVAL, "unknown system");
    if (p->scheme < COLA_CG_FP64 || p->scheme > COLA_CG_FP32_DEFECT)
        return set_error(h, COLA_EINVAL, "unknown scheme");
    if (!(p->tol > 0) || p->max_iter < 1) return set_error(h, COLA_EINVAL, "bad tol / max_iter");
    if (p->block && (p->system == COLA_SYS_MDAGM ||
                     (p->scheme != COLA_CG_FP16_DEFECT && p->scheme != COLA_CG_FP32_DEFECT)))
        return set_error(h, COLA_EINVAL,
                         "block CG runs as the inner solver of the defect-correction schemes on "
                         "the even-odd systems");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    if (p->scheme != COLA_CG_FP64 && !h->su3)
        return set_error(h, COLA_EINVAL, "mixed-precision schemes need an SU(3) gauge field");
    return cg_solve_impl(h, x, b, nrhs, p, r, as_stream(stream));
}

int cola_cg_multishift(cola_handle_t *h, void *x, const void *b, int nshift, const double *shifts,
                       const cola_cg_params_t *p, cola_cg_result_t *r, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!x || !b || !p || !shifts) return set_error(h, COLA_EINVAL, "null pointer");
    if (nshift < 1 || nshift > kMaxRhs)
        return set_error(h, COLA_EINVAL, "nshift must be 1 .. 16");
    for (int q = 0; q < nshift; ++q)
        if (!(shifts[q] >= 0.0) || !std::isfinite(shifts[q]))
            return set_error(h, COLA_EINVAL, "shifts must be finite and >= 0");
    if (p->system != COLA_SYS_MDAGM && p->system != COLA_SYS_SCHUR)
        return set_error(h, COLA_EINVAL, "multi-shift CG runs on the MDAGM and SCHUR systems");
    if (p->scheme != COLA_CG_FP64 || p->block)
        return set_error(h, COLA_EINVAL, "multi-shift CG is FP64, lockstep");
    if (!(p->tol > 0) || p->max_iter < 1) return set_error(h, COLA_EINVAL, "bad tol / max_iter");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    return cg_multishift_impl(h, x, b, nshift, shifts, p, r, as_stream(stream));
}

int cola_eigensolve(cola_handle_t *h, void *X, int n, const cola_eig_params_t *p,
                    cola_eig_result_t *r, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!X || !p) return set_error(h, COLA_EINVAL, "null pointer");
    if (n < 1 || n > kEigMax) return set_error(h, COLA_EINVAL, "n must be 1 .. 32");
    if (p->system != COLA_SYS_MDAGM && p->system != COLA_SYS_SCHUR)
        return set_error(h, COLA_EINVAL, "the eigensolver runs on the MDAGM and SCHUR systems");
    if (!(p->tol > 0)) return set_error(h, COLA_EINVAL, "tol must be > 0");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    return eigensolve_impl(h, X, n, p, r, as_stream(stream));
}

int cola_cg_deflated(cola_handle_t *h, void *x, const void *b, int nrhs, const void *X,
                     const double *lambda, int n, const cola_cg_params_t *p,
                     cola_cg_result_t *r, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!x || !b || !X || !lambda || !p) return set_error(h, COLA_EINVAL, "null pointer");
    if (x == b) return set_error(h, COLA_EINVAL, "x and b must not overlap");
    COLA_TRY(check_rhs(h, nrhs));
    if (n < 1 || n > kEigMax) return set_error(h, COLA_EINVAL, "n must be 1 .. 32");
    for (int i = 0; i < n; ++i)
        if (!(lambda[i] > 0) || !std::isfinite(lambda[i]))
            return set_error(h, COLA_EINVAL, "eigenvalues must be finite and > 0");
    if (p->system != COLA_SYS_MDAGM && p->system != COLA_SYS_SCHUR)
        return set_error(h, COLA_EINVAL, "deflated CG runs on the MDAGM and SCHUR systems");
    if (p->scheme < COLA_CG_FP64 || p->scheme > COLA_CG_FP32_DEFECT)
        return set_error(h, COLA_EINVAL, "unknown scheme");
    if (!(p->tol > 0) || p->max_iter < 1) return set_error(h, COLA_EINVAL, "bad tol / max_iter");
    if (p->block && (p->system != COLA_SYS_SCHUR || (p->scheme != COLA_CG_FP16_DEFECT &&
                                                     p->scheme != COLA_CG_FP32_DEFECT)))
        return set_error(h, COLA_EINVAL, "block CG needs a DEFECT scheme on the SCHUR system");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    if (p->scheme != COLA_CG_FP64 && !h->su3)
        return set_error(h, COLA_EINVAL, "mixed schemes need an SU(3) gauge field");
    return cg_deflated_impl(h, x, b, nrhs, X, lambda, n, p, r, as_stream(stream));
}

int cola_fermion_force(cola_handle_t *h, void *F, const void *X, const void *Y, int mode,
                       void *stream) {
    if (!h) return COLA_EINVAL;
    if (!F || !X || !Y) return set_error(h, COLA_EINVAL, "null pointer");
    if (mode != COLA_FORCE_GRAD && mode != COLA_FORCE_LIE)
        return set_error(h, COLA_EINVAL, "unknown force mode");
    if (h->csw != 0.0) return set_error(h, COLA_EINVAL, "force of the clover term not available");
    if (h->flic) return set_error(h, COLA_EINVAL, "force of the FLIC operator not available");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    COLA_HIP(h, launch_force(h->g, h->gauge[0], X, Y, F, h->kappa, h->phase, mode,
                             as_stream(stream)));
    return COLA_OK;
}

int cola_get_stats(cola_handle_t *h, cola_stats_t *s) {
    if (!h || !s) return COLA_EINVAL;
    COLA_TRY(flush_timing(h, true));
    *s = h->stats;
    return COLA_OK;
}

int cola_reset_stats(cola_handle_t *h) {
    if (!h) return COLA_EINVAL;
    COLA_TRY(flush_timing(h, true));
    memset(&h->stats, 0, sizeof h->stats);
    return COLA_OK;
}

int cola_set_tuning(cola_handle_t *h, int mode) {
    if (!h || mode < 0 || mode > 2) return COLA_EINVAL;
    h->tune_mode = mode;
    return COLA_OK;
}

int cola_tune_load(cola_handle_t *h, const char *path) {
    if (!h) return COLA_EINVAL;
    return tune_cache_load(h, path);
}

int cola_tune_save(cola_handle_t *h, const char *path) {
    if (!h) return COLA_EINVAL;
    return tune_cache_save(h, path);
}

size_t cola_tune_dump(const cola_handle_t *h, char *buf, size_t len) {
    if (!h) return 0;
    std::string s = "{";
    bool first = true;
    for (auto &kv : h->tune) {
        char e[256];
        snprintf(e, sizeof e,
                 "%s\"%s\": {\"rpt\": %d, \"sites_per_block\": %d, \"grid\": %d, "
                 "\"tchunk\": %d, \"tile\": [%d, %d], \"stage_links\": %d, \"ms\": %.6f}",
                 first ? "" : ", ", kv.first.c_str(), kv.second.rpt, kv.second.sites_per_block,
                 kv.second.grid, kv.second.tchunk, kv.second.tile_y, kv.second.tile_z,
                 kv.second.stage, kv.second.ms);
        s += e;
        first = false;
    }
    s += "}";
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, s.size());
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return s.size() + 1;
}

}  // extern "C"
