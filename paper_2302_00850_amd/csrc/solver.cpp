// Conjugate-gradient solvers on the normal operator (M^H M on the full lattice
// or S^H S on even sites), built from the hop and site kernels.
//
// All right-hand sides advance in lockstep (one batched hop per operator
// factor).  Per-rhs scalars (rho, pi, alpha, beta) live on the device; the
// host reads the residual norms back every `check_interval` iterations only.
//
// Schemes (the paper's benchmark is a mixed-precision solver with 32-bit
// inner iterations and a 64-bit outer solver):
//   FP64          plain CG; when the iterated residual meets tol the true
//                 residual b - A x is recomputed and CG continues from it if
//                 needed.
//   FP32_RELIABLE FP32 CG (FP32 vectors, 12-real FP32 links) with an FP64
//                 solution accumulator: every reliable_interval iterations
//                 (and when the iterated residual meets tol) x64 += x32,
//                 r = b - A64 x64 in FP64, and the FP32 residual is replaced;
//                 the search direction is kept.
//   FP16/FP32_DEFECT  FP64 defect correction: R = B - A64 X, inner CG on
//                 A E = R/|R| in FP16 storage (FP32 arithmetic) or FP32 down
//                 to inner_tol, X += |R| E.  Three cycles that contract the
//                 residual by less than 2x switch an FP16 inner solve to FP32.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "handle.h"

namespace cola {

namespace {

enum Slot {
    RHO = 0,
    RHO_NEW = 1,
    PI = 2,
    PI2 = 3,
    BNORM = 4,
    SCALE = 5,
    TRUE_RES = 6,
    TMP = 7,
    RHO_EVEN = 8  // |r|^2 of the even block (full-lattice fused CG step)
};

struct Ctx {
    cola_handle_t *h;
    hipStream_t st;
    int R;
    int full;  // 1: M^H M on the full lattice (2 blocks), 0: S^H S on even sites
    int nblk() const { return full ? 2 : 1; }
    size_t bytes(SpinorFmt f) const { return spinor_block_bytes(h->g, f, R) * nblk(); }
    BlasShape shape() const { return blas_shape(h->g, R, nblk()); }
    double *slot(int s) const { return scal_slot(h, s); }
};

// Iterations between host convergence checks when the caller leaves it to the library.
// A check reads the residual norms back and waits for them (some 10-20 us during which
// the device idles), and the solve stops only at a check, overshooting by up to
// check - 1 iterations.  Where an iteration moves at least 2^20 site-rhs through the
// operator (a millisecond or more) the wait costs under 2% and every iteration is
// checked; smaller solves check every `small` iterations.
int default_check(const Ctx &c, int small) {
    const double work = (double)c.h->g.Vh * c.R * c.nblk();
    return work >= 1048576.0 ? 1 : small;
}

int vec(const Ctx &c, const char *tag, SpinorFmt f, void **out) {
    std::string t = std::string("cg_") + tag + "_" + std::to_string((int)f) + "_" +
                    std::to_string(c.R) + "_" + std::to_string(c.full);
    return get_vec(c.h, t, c.bytes(f), out);
}

// out = A in, |first factor output|^2 -> PI (+PI2 on the full lattice)
int normal(const Ctx &c, int prec, void *out, const void *in) {
    if (!c.full)
        return apply_op(c.h, out, in, COLA_OP_SCHUR_DAGSCHUR, 0, prec, c.R, c.st, c.slot(PI));
    cola_handle_t *h = c.h;
    const SpinorFmt sf = spinor_fmt(prec);
    const size_t bb = spinor_block_bytes(h->g, sf, c.R);
    void *t;
    COLA_TRY(get_vec(h, "cg_full_t_" + std::to_string((int)sf) + "_" + std::to_string(c.R),
                     2 * bb, &t));
    const bool clover = h->csw != 0.0;
    const void *A = sf == SpinorFmt::F64 ? h->clov64 : h->clov32;
    for (int p = 0; p < 2; ++p) {
        HopCall hc{(char *)t + p * bb, (const char *)in + (1 - p) * bb, p, 0};
        hc.epi = clover ? EPI_CLOV_XPAY : EPI_XPAY;
        hc.x = (const char *)in + p * bb;
        hc.a = -h->kappa;
        hc.clov = A;
        hc.norm_result = c.slot(p == 0 ? PI : PI2);
        COLA_TRY(hop(h, hc, prec, c.R, c.st));
    }
    return apply_op(h, out, t, COLA_OP_MDAG, -1, prec, c.R, c.st);
}

// One CG step: Ap = A p, pi = <p, Ap>, then x += alpha p, r -= alpha Ap and
// rho_new = |r|^2.  With x, r and p in the operator's storage the update runs inside the
// last hops (Ap is never stored): the last hop of S^dag S on the even-odd system, the two
// parity hops of M^dag on the full lattice; COLA_CG_FUSE=0 selects the separate update
// kernel.
int full_normal_cg_step(const Ctx &c, int prec, void *x, void *r, void *pv) {
    cola_handle_t *h = c.h;
    const SpinorFmt sf = spinor_fmt(prec);
    const size_t bb = spinor_block_bytes(h->g, sf, c.R);
    void *t;
    COLA_TRY(get_vec(h, "cg_full_t_" + std::to_string((int)sf) + "_" + std::to_string(c.R),
                     2 * bb, &t));
    const bool clover = h->csw != 0.0;
    const void *A = sf == SpinorFmt::F64 ? h->clov64 : h->clov32;
    auto blk = [bb](const void *base, int q) { return (char *)base + q * bb; };
    // t = M p, |t_e|^2 -> PI, |t_o|^2 -> PI2
    for (int q = 0; q < 2; ++q) {
        HopCall hc{blk(t, q), blk(pv, 1 - q), q, 0};
        hc.epi = clover ? EPI_CLOV_XPAY : EPI_XPAY;
        hc.x = blk(pv, q);
        hc.a = -h->kappa;
        hc.clov = A;
        hc.norm_result = c.slot(q == 0 ? PI : PI2);
        COLA_TRY(hop(h, hc, prec, c.R, c.st));
    }
    // per parity: the M^dag hop with the update of x and r; |r_e|^2 + |r_o|^2 -> RHO_NEW
    for (int q = 0; q < 2; ++q) {
        HopCall hc{blk(r, q), blk(t, 1 - q), q, 1};
        hc.epi = clover ? EPI_CLOV_XPAY_CG : EPI_XPAY_CG;
        hc.x = blk(t, q);
        hc.a = -h->kappa;
        hc.clov = A;
        hc.norm_result = c.slot(q == 0 ? RHO_EVEN : RHO_NEW);
        hc.cg_x = blk(x, q);
        hc.cg_r = blk(r, q);
        hc.cg_p = blk(pv, q);
        hc.cg_rho = c.slot(RHO);
        hc.cg_pi = c.slot(PI);
        hc.cg_pi2 = c.slot(PI2);
        hc.cg_active = h->active;
        COLA_TRY(hop(h, hc, prec, c.R, c.st));
    }
    COLA_HIP(h, launch_scalar_add(c.slot(RHO_NEW), c.slot(RHO_EVEN), c.R, c.st));
    return COLA_OK;
}

int cg_step(const Ctx &c, int prec, SpinorFmt fx, void *x, void *r, void *pv, void *ap) {
    cola_handle_t *h = c.h;
    const SpinorFmt fp = spinor_fmt(prec);
    const char *env = getenv("COLA_CG_FUSE");
    const bool fuse = fx == fp && !(env && env[0] == '0');
    if (fuse && c.full) return full_normal_cg_step(c, prec, x, r, pv);
    if (fuse)
        return schur_normal_cg_step(h, prec, c.R, c.st, x, r, pv, c.slot(RHO), c.slot(PI),
                                    h->active, c.slot(RHO_NEW));
    COLA_TRY(normal(c, prec, ap, pv));
    COLA_HIP(h, launch_cg_xr(c.shape(), fx, fp, fx, fp, x, pv, r, ap, c.slot(RHO), c.slot(PI),
                             c.full ? c.slot(PI2) : nullptr, h->active,
                             reduce_into(h, RHO_NEW), c.st));
    return COLA_OK;
}

int zero_pi2(const Ctx &c) {
    COLA_HIP(c.h, hipMemsetAsync(c.slot(PI2), 0, sizeof(double) * kMaxRhs, c.st));
    return COLA_OK;
}

// r = b - A x in FP64 (x may be all zero); |r|^2 -> slot
int true_residual(const Ctx &c, void *r, const void *b, const void *x, int slot) {
    void *ax;
    COLA_TRY(vec(c, "ax64", SpinorFmt::F64, &ax));
    COLA_TRY(normal(c, COLA_FP64, ax, x));
    const Reduce red = reduce_into(c.h, slot);
    COLA_HIP(c.h, launch_residual(c.shape(), r, b, ax, red, c.st));
    return COLA_OK;
}

// The starting residual: b - A x, or b itself (and |b|^2, already in BNORM) when the
// solve starts from x = 0, which saves the four FP64 hops of the normal operator.
int initial_residual(const Ctx &c, void *r, const void *b, const void *x, bool x_zero) {
    if (!x_zero) return true_residual(c, r, b, x, TRUE_RES);
    COLA_HIP(c.h, hipMemcpyAsync(r, b, c.bytes(SpinorFmt::F64), hipMemcpyDeviceToDevice, c.st));
    COLA_HIP(c.h, hipMemcpyAsync(c.slot(TRUE_RES), c.slot(BNORM), sizeof(double) * c.R,
                                 hipMemcpyDeviceToDevice, c.st));
    return COLA_OK;
}

int read_slot(const Ctx &c, int slot, double *out) {
    COLA_HIP(c.h, hipMemcpyAsync(out, c.slot(slot), sizeof(double) * c.R, hipMemcpyDeviceToHost,
                                 c.st));
    COLA_HIP(c.h, hipStreamSynchronize(c.st));
    return COLA_OK;
}

int write_active(const Ctx &c, const std::vector<int> &act) {
    memcpy(c.h->host_active, act.data(), sizeof(int) * c.R);
    COLA_HIP(c.h, hipMemcpyAsync(c.h->active, c.h->host_active, sizeof(int) * c.R,
                                 hipMemcpyHostToDevice, c.st));
    COLA_HIP(c.h, hipStreamSynchronize(c.st));  // the pinned staging area is reused
    return COLA_OK;
}

int write_slot(const Ctx &c, int slot, const std::vector<double> &v) {
    std::vector<double> tmp(v);
    COLA_HIP(c.h, hipMemcpyAsync(c.slot(slot), tmp.data(), sizeof(double) * c.R,
                                 hipMemcpyHostToDevice, c.st));
    COLA_HIP(c.h, hipStreamSynchronize(c.st));
    return COLA_OK;
}

bool finite_all(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// swap the RHO and RHO_NEW slots by copying (keeps slot numbering fixed); a kernel, so
// that captured iteration blocks hold kernel nodes only
int rotate_rho(const Ctx &c) {
    COLA_HIP(c.h, launch_scalar_copy(c.slot(RHO), c.slot(RHO_NEW), c.R, c.st));
    return COLA_OK;
}

struct Outcome {
    int status = COLA_OK;
    int iterations = 0;
    int outer = 0;
    int reliable = 0;
    std::vector<double> final_tr;  // true |r|^2 of the returned x, when the solver has it
};

// ---------------------------------------------------------------- iteration blocks

// Small solves are bound by launch latency (a 16^3 x 32 CG iteration runs ~90 us of
// kernels in ~165 us), so with COLA_GRAPHS=1 the n iterations between two convergence
// checks -- (step, p update, rho rotation) x (n - 1), step -- are captured once as a HIP
// graph and replayed (large solves check every iteration and launch directly).  Capture
// needs every launch shape settled (the first block of a solve runs directly, which
// tunes) and no per-launch timing.  Off by default: measured on 16^3 x 32 and 8^3 x 16,
// the replays ran 4-10% slower than the direct launches.
bool graphs_wanted(const Ctx &c) {
    const char *env = getenv("COLA_GRAPHS");
    if (!env || env[0] != '1') return false;
    if ((c.h->flags & COLA_FLAG_TIMING) || c.h->tune_mode == 2) return false;
    return (double)c.h->g.Vh * c.R * c.nblk() < 1048576.0;
}

int cg_block(const Ctx &c, int prec, SpinorFmt fx, void *x, void *r, void *pv, void *ap, int n,
             bool graph) {
    cola_handle_t *h = c.h;
    const SpinorFmt fp = spinor_fmt(prec);
    auto body = [&](const Ctx &cc) -> int {
        for (int k = 0; k < n; ++k) {
            COLA_TRY(cg_step(cc, prec, fx, x, r, pv, ap));
            if (k + 1 < n) {
                COLA_HIP(h, launch_cg_p(cc.shape(), fx, fp, r, pv, cc.slot(RHO_NEW),
                                        cc.slot(RHO), h->active, cc.st));
                COLA_TRY(rotate_rho(cc));
            }
        }
        return COLA_OK;
    };
    if (!graph || n < 2) return body(c);
    if (!h->gstream) {
        COLA_HIP(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        COLA_HIP(h, hipEventCreateWithFlags(&h->gevent, hipEventDisableTiming));
    }
    // everything the captured launches hold: vectors, fields, operator, shape
    char key[512];
    const char *fuse = getenv("COLA_CG_FUSE");
    snprintf(key, sizeof key, "%d %d %d %d %d %p %p %p %p %p %p %p %p %p %p %p %p %p %p %p %p %d %c",
             prec, (int)fx, c.R, c.full, n, x, r, pv, ap, h->gauge[0], h->gauge[1], h->gauge[2],
             h->gauge[3], h->fat[0], h->fat[1], h->fat[2], h->fat[3], h->clov32, h->clov64,
             h->clovinv32, h->clovinv64, h->flic ? 1 : 0, fuse ? fuse[0] : '-');
    hipGraphExec_t exec;
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        exec = it->second;
    } else {
        Ctx cg = c;
        cg.st = h->gstream;
        COLA_HIP(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeRelaxed));
        const int rc = body(cg);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->gstream, &graph);
        if (rc != COLA_OK) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        COLA_HIP(h, ec);
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        COLA_HIP(h, ei);
        h->graphs[key] = exec;
    }
    // ordered after the caller's stream, and the caller's stream after it
    COLA_HIP(h, hipEventRecord(h->gevent, c.st));
    COLA_HIP(h, hipStreamWaitEvent(h->gstream, h->gevent, 0));
    COLA_HIP(h, hipGraphLaunch(exec, h->gstream));
    COLA_HIP(h, hipEventRecord(h->gevent, h->gstream));
    COLA_HIP(h, hipStreamWaitEvent(c.st, h->gevent, 0));
    return COLA_OK;
}

}  // namespace

void graphs_clear(cola_handle_t *h) {
    for (auto &kv : h->graphs) hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

namespace {

// ---------------------------------------------------------------- FP64 / FP32 reliable

int solve_reliable(const Ctx &c, int sloppy_prec, const cola_cg_params_t &p, void *x64,
                   const void *b64, const std::vector<double> &thr, Outcome *o) {
    const bool x_zero = !p.use_x0;
    cola_handle_t *h = c.h;
    const BlasShape sh = c.shape();
    const SpinorFmt fs = spinor_fmt(sloppy_prec);
    const bool same = fs == SpinorFmt::F64;
    const int check = p.check_interval > 0 ? p.check_interval : default_check(c, same ? 8 : 5);
    const int interval = same ? (1 << 30) : std::max(1, p.reliable_interval);
    // also update once the iterated residual has fallen by delta since the last
    // update (Clark et al.): a sloppy residual far below the true one would make
    // beta = rho_true / rho_iter huge and leave p pointing the stale way
    const double delta2 = 1e-2;
    void *r64, *xs, *rs, *ps, *aps;
    COLA_TRY(vec(c, "r64", SpinorFmt::F64, &r64));
    COLA_TRY(vec(c, "ps", fs, &ps));
    COLA_TRY(vec(c, "aps", fs, &aps));
    if (same) {
        xs = x64;
        rs = r64;
    } else {
        COLA_TRY(vec(c, "xs", fs, &xs));
        COLA_TRY(vec(c, "rs", fs, &rs));
        COLA_HIP(h, hipMemsetAsync(xs, 0, c.bytes(fs), c.st));
    }
    // r = b - A x0, rho = |r|^2
    COLA_TRY(initial_residual(c, r64, b64, x64, x_zero));
    std::vector<double> rho(c.R), tr(c.R);
    COLA_TRY(read_slot(c, TRUE_RES, tr.data()));
    if (!finite_all(tr.data(), c.R)) {
        o->status = COLA_BREAKDOWN;
        return COLA_OK;
    }
    std::vector<int> act(c.R);
    std::vector<double> ref(tr);  // true |r|^2 at the last reliable update
    bool all_done = true;
    for (int q = 0; q < c.R; ++q) {
        act[q] = tr[q] > thr[q];
        all_done &= !act[q];
    }
    if (all_done) {
        o->final_tr = tr;
        return COLA_OK;
    }
    COLA_TRY(write_active(c, act));
    const Reduce red_rho = reduce_into(h, RHO);
    if (!same) COLA_HIP(h, launch_convert(sh, fs, SpinorFmt::F64, rs, r64, nullptr, 0, &red_rho, c.st));
    else COLA_HIP(h, hipMemcpyAsync(c.slot(RHO), c.slot(TRUE_RES), sizeof(double) * c.R, hipMemcpyDeviceToDevice, c.st));
    COLA_HIP(h, launch_convert(sh, fs, fs, ps, rs, nullptr, 0, nullptr, c.st));
    if (!c.full) COLA_TRY(zero_pi2(c));
    const Reduce red_new = reduce_into(h, RHO_NEW);
    int last_rel = 0;
    int it = 0;
    const bool graphs = graphs_wanted(c);
    while (it < p.max_iter) {
        // the iterations up to the next check (it % check == 0 or the cap)
        const int n = std::min(check - it % check, p.max_iter - it);
        COLA_TRY(cg_block(c, sloppy_prec, fs, xs, rs, ps, aps, n, graphs && it > 0));
        it += n;
        bool stop = false;
        {
            COLA_TRY(read_slot(c, RHO_NEW, rho.data()));
            if (!finite_all(rho.data(), c.R)) {
                o->status = COLA_BREAKDOWN;
                break;
            }
            bool iter_conv = true, dropped = false;
            for (int q = 0; q < c.R; ++q) {
                iter_conv &= !act[q] || rho[q] <= thr[q];
                dropped |= act[q] && rho[q] < delta2 * ref[q];
            }
            if (iter_conv || dropped || it - last_rel >= interval || it == p.max_iter) {
                if (!same) {
                    COLA_HIP(h, launch_accum(sh, fs, x64, xs, nullptr, 1, c.st));
                }
                COLA_TRY(true_residual(c, r64, b64, x64, TRUE_RES));
                COLA_TRY(read_slot(c, TRUE_RES, tr.data()));
                ++o->reliable;
                last_rel = it;
                bool done = true, restart = false;
                std::vector<int> keep(c.R);
                for (int q = 0; q < c.R; ++q) {
                    act[q] = tr[q] > thr[q];
                    done &= !act[q];
                    ref[q] = tr[q];
                    // true residual far above the iterated one: restart p = r
                    keep[q] = act[q] && !(tr[q] > 1e4 * rho[q]);
                    restart |= act[q] && !keep[q];
                }
                if (done) {
                    stop = true;
                    o->final_tr = tr;  // x64 holds the whole solution (xs was folded in)
                } else {
                    if (!same)
                        COLA_HIP(h, launch_convert(sh, fs, SpinorFmt::F64, rs, r64, nullptr, 0,
                                                   &red_new, c.st));
                    else
                        COLA_HIP(h, hipMemcpyAsync(c.slot(RHO_NEW), c.slot(TRUE_RES),
                                                   sizeof(double) * c.R, hipMemcpyDeviceToDevice,
                                                   c.st));
                    if (restart) {
                        // beta = 0 for the restarted columns: p = r
                        COLA_TRY(write_active(c, keep));
                        COLA_HIP(h, launch_cg_p(sh, fs, fs, rs, ps, c.slot(RHO_NEW), c.slot(RHO),
                                                h->active, c.st));
                        COLA_TRY(rotate_rho(c));
                        COLA_TRY(write_active(c, act));
                        continue;
                    }
                    COLA_TRY(write_active(c, act));
                }
            }
        }
        if (stop) break;
        COLA_HIP(h, launch_cg_p(sh, fs, fs, rs, ps, c.slot(RHO_NEW), c.slot(RHO), h->active, c.st));
        COLA_TRY(rotate_rho(c));
    }
    if (!same && o->status == COLA_OK) {
        // fold any remaining sloppy solution in (no-op after a final reliable update)
        COLA_HIP(h, launch_accum(sh, fs, x64, xs, nullptr, 1, c.st));
    }
    o->iterations += it;
    if (o->status == COLA_OK && it >= p.max_iter) {
        COLA_TRY(true_residual(c, r64, b64, x64, TRUE_RES));
        COLA_TRY(read_slot(c, TRUE_RES, tr.data()));
        for (int q = 0; q < c.R; ++q)
            if (tr[q] > thr[q]) o->status = COLA_NOT_CONVERGED;
        o->final_tr = tr;
    }
    return COLA_OK;
}

// ---------------------------------------------------------------- defect correction

// CG iterations on the normal system in precision prec (p, Ap in that storage; x and r
// in storage fx, FP32 arithmetic throughout).
int inner_cg(const Ctx &c, int prec, SpinorFmt fx, void *x, void *r, void *pv, void *ap,
             const std::vector<double> &inner_tol2, int max_it, std::vector<int> act, int check,
             int *iters, int *status) {
    cola_handle_t *h = c.h;
    const BlasShape sh = c.shape();
    const SpinorFmt fp = spinor_fmt(prec);
    COLA_TRY(write_active(c, act));
    std::vector<double> rho(c.R);
    int it = 0;
    const bool graphs = graphs_wanted(c);
    while (it < max_it) {
        // the iterations up to the next check
        const int n = std::min(check - it % check, max_it - it);
        COLA_TRY(cg_block(c, prec, fx, x, r, pv, ap, n, graphs && it > 0));
        it += n;
        if (it % check == 0) {
            COLA_TRY(read_slot(c, RHO_NEW, rho.data()));
            if (!finite_all(rho.data(), c.R)) {
                *status = COLA_BREAKDOWN;
                break;
            }
            bool any = false;
            for (int q = 0; q < c.R; ++q) {
                if (act[q] && rho[q] <= inner_tol2[q]) act[q] = 0;
                any |= act[q] != 0;
            }
            if (!any) break;
            COLA_TRY(write_active(c, act));
        }
        COLA_HIP(h, launch_cg_p(sh, fx, fp, r, pv, c.slot(RHO_NEW), c.slot(RHO), h->active, c.st));
        COLA_TRY(rotate_rho(c));
    }
    *iters = it;
    return COLA_OK;
}

// ---------------------------------------------------------------- block CG

// O'Leary block CG on A E = R (R given in r32, E accumulated in x32), all active
// columns sharing one Krylov space, A = S^H S on the even sites:
//   T = S P, Q = S^H T; alpha = (T^H T)^-1 (R^H R); E += P alpha; R -= Q alpha;
//   beta = (R^H R)_old^-1 (R^H R)_new; P = R + P beta.
// P^H Q is taken as T^H T (the same matrix, Hermitian positive semi-definite by
// construction, and one field read instead of two).  The Gram matrices and the two small
// Hermitian solves (Cholesky with deflation of dependent directions, block_solve_kernel)
// stay on the device; R^H R comes out of the update kernel itself.  The host reads the
// diagonal of R^H R every `check` iterations to stop once every active column's
// |R_q|^2 <= inner_tol2 (the columns start at 1).
int inner_block_cg(const Ctx &c, int prec, void *x32, void *r32,
                   const std::vector<double> &inner_tol2, int max_it, std::vector<int> act,
                   int check, int *iters, int *status) {
    cola_handle_t *h = c.h;
    const int n = c.R;
    const SpinorFmt fp = spinor_fmt(prec);
    const SpinorFmt fx = SpinorFmt::F32;
    const int S = h->g.S;
    void *P, *Pn, *Q, *T, *mats;
    COLA_TRY(vec(c, "bP", fp, &P));
    COLA_TRY(vec(c, "bPn", fp, &Pn));
    COLA_TRY(vec(c, "bQ", fp, &Q));
    COLA_TRY(vec(c, "bT", fp, &T));
    // five n x n complex matrices: T^H T, R^H R (two, alternating), alpha, beta
    const size_t mat = (size_t)2 * kMaxRhs * kMaxRhs;
    COLA_TRY(get_vec(h, "block_mats", sizeof(double) * 5 * mat, &mats));
    double *Gpi = (double *)mats, *Grho[2] = {Gpi + mat, Gpi + 2 * mat}, *alpha = Gpi + 3 * mat,
           *beta = Gpi + 4 * mat;
    std::vector<double> host(2 * (size_t)n * n);
    unsigned mask_bits = 0;
    // inactive columns take no part: zero their residual so they stay at E = 0
    std::vector<double> mask(n);
    for (int q = 0; q < n; ++q) {
        mask[q] = act[q] ? 1.0 : 0.0;
        if (act[q]) mask_bits |= 1u << q;
    }
    COLA_TRY(write_slot(c, TMP, mask));
    const BlasShape sh = c.shape();
    COLA_HIP(h, launch_convert(sh, fx, fx, r32, r32, c.slot(TMP), 0, nullptr, c.st));
    COLA_HIP(h, launch_convert(sh, fp, fx, P, r32, nullptr, 0, nullptr, c.st));
    auto red = [&](double *out) { return Reduce{h->partial, h->counter, out}; };
    int cur = 0;
    COLA_HIP(h, launch_gram(S, n, h->num_cu, fx, fx, r32, r32, red(Grho[cur]), c.st));
    int it = 0;
    while (it < max_it) {
        COLA_TRY(apply_op(h, T, P, COLA_OP_SCHUR, 0, prec, n, c.st));
        COLA_HIP(h, launch_gram(S, n, h->num_cu, fp, fp, T, T, red(Gpi), c.st));
        COLA_TRY(apply_op(h, Q, T, COLA_OP_SCHUR_DAG, 0, prec, n, c.st));
        COLA_HIP(h, launch_block_solve(Gpi, Grho[cur], mask_bits, n, alpha, c.st));
        const Reduce rr = red(Grho[1 - cur]);
        COLA_HIP(h, launch_block_axpy(S, n, h->num_cu, fx, fp, x32, P, r32, Q, alpha, &rr,
                                      c.st));
        ++it;
        if (it % check == 0 || it == max_it) {
            COLA_HIP(h, hipMemcpyAsync(host.data(), Grho[1 - cur], sizeof(double) * host.size(),
                                       hipMemcpyDeviceToHost, c.st));
            COLA_HIP(h, hipStreamSynchronize(c.st));
            bool any = false, bad = false;
            for (int q = 0; q < n; ++q) {
                const double d = host[2 * (q * n + q)];  // (R^H R)_qq
                bad |= !std::isfinite(d);
                any |= act[q] && d > inner_tol2[q];
            }
            if (bad) {
                *status = COLA_BREAKDOWN;
                break;
            }
            if (!any) break;
        }
        COLA_HIP(h, launch_block_solve(Grho[cur], Grho[1 - cur], mask_bits, n, beta, c.st));
        COLA_HIP(h, launch_block_xpay(S, n, h->num_cu, fx, fp, Pn, r32, P, beta, c.st));
        std::swap(P, Pn);
        cur = 1 - cur;
    }
    *iters = it;
    return COLA_OK;
}

int solve_defect(const Ctx &c, int inner_prec, const cola_cg_params_t &p, void *x64,
                 const void *b64, const std::vector<double> &thr, Outcome *o) {
    cola_handle_t *h = c.h;
    const BlasShape sh = c.shape();
    const int check = p.check_interval > 0 ? p.check_interval : default_check(c, 8);
    // default inner reductions: about as deep as the inner storage keeps the iterated
    // residual honest (FP16 ~5e-4 per rounding, FP32 ~6e-8), so that few restarts throw
    // away Krylov spaces: FP16 1e-2, FP32 1e-5 (two cycles for a 1e-10 solve)
    const double itol = p.inner_tol > 0 ? p.inner_tol : (inner_prec == COLA_FP16 ? 1e-2 : 1e-5);
    void *r64, *x32, *r32;
    COLA_TRY(vec(c, "r64", SpinorFmt::F64, &r64));
    COLA_TRY(vec(c, "x32", SpinorFmt::F32, &x32));
    COLA_TRY(vec(c, "r32", SpinorFmt::F32, &r32));
    std::vector<double> tr(c.R), prev(c.R, -1.0), s(c.R);
    int slow = 0;
    int prec = inner_prec;
    while (true) {
        COLA_TRY(initial_residual(c, r64, b64, x64, !p.use_x0 && o->outer == 0));
        COLA_TRY(read_slot(c, TRUE_RES, tr.data()));
        if (!finite_all(tr.data(), c.R)) {
            o->status = COLA_BREAKDOWN;
            return COLA_OK;
        }
        std::vector<int> act(c.R);
        bool done = true;
        double worst = 0;
        for (int q = 0; q < c.R; ++q) {
            act[q] = tr[q] > thr[q];
            done &= !act[q];
            s[q] = std::sqrt(tr[q]);
            if (act[q] && prev[q] > 0) worst = std::max(worst, std::sqrt(tr[q] / prev[q]));
        }
        if (done) {
            o->final_tr = tr;
            return COLA_OK;
        }
        if (o->iterations >= p.max_iter) {
            o->status = COLA_NOT_CONVERGED;
            return COLA_OK;
        }
        // Inner target per column (relative to |R|): the scheme's reduction, relaxed to
        // ten times below what the column still needs so the last cycle does not solve
        // far past the tolerance.
        std::vector<double> itol2(c.R, itol * itol);
        for (int q = 0; q < c.R; ++q)
            if (act[q] && tr[q] > 0) itol2[q] = std::max(itol * itol, 1e-2 * thr[q] / tr[q]);
        if (o->outer > 0 && worst > 0.5) {
            if (++slow >= 3 && prec == COLA_FP16) {
                prec = COLA_FP32;
                slow = 0;
            }
        } else {
            slow = 0;
        }
        prev = tr;
        COLA_TRY(write_slot(c, SCALE, s));
        const SpinorFmt fp = spinor_fmt(prec);
        void *pv, *ap;
        COLA_TRY(vec(c, "dp", fp, &pv));
        COLA_TRY(vec(c, "dap", fp, &ap));
        const Reduce red_rho = reduce_into(h, RHO);
        // Inner vectors: r = R / |R| (rho = |r|^2), p = r, x = 0.  Block CG keeps x and r in
        // FP32; the lockstep solver stores them like p, in the inner precision (FP16 rounds
        // them to about 5e-4 per update, far below the inner solve's 1e-2 reduction, and
        // saves a third of the bytes of the update kernels).
        const SpinorFmt fxr = p.block ? SpinorFmt::F32 : fp;
        void *xs = x32, *rs = r32;
        if (fxr != SpinorFmt::F32) {
            COLA_TRY(vec(c, "dx", fxr, &xs));
            COLA_TRY(vec(c, "dr", fxr, &rs));
        }
        COLA_HIP(h, launch_convert(sh, fxr, SpinorFmt::F64, rs, r64, c.slot(SCALE), 1, &red_rho,
                                   c.st));
        COLA_HIP(h, launch_convert(sh, fp, fxr, pv, rs, nullptr, 0, nullptr, c.st));
        COLA_HIP(h, hipMemsetAsync(xs, 0, c.bytes(fxr), c.st));
        if (!c.full) COLA_TRY(zero_pi2(c));
        int its = 0, st = COLA_OK;
        if (p.block)
            COLA_TRY(inner_block_cg(c, prec, x32, r32, itol2, p.max_iter - o->iterations, act,
                                    check, &its, &st));
        else
            COLA_TRY(inner_cg(c, prec, fxr, xs, rs, pv, ap, itol2, p.max_iter - o->iterations,
                              act, check, &its, &st));
        o->iterations += its;
        ++o->outer;
        if (st != COLA_OK) {
            o->status = st;
            return COLA_OK;
        }
        // X += |R| E
        COLA_HIP(h, launch_accum(sh, fxr, x64, xs, c.slot(SCALE), 0, c.st));
    }
}

}  // namespace

int cg_solve_impl(cola_handle_t *h, void *x, const void *b, int nrhs, const cola_cg_params_t *p,
                  cola_cg_result_t *r, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    Ctx c{h, st, nrhs, p->system == COLA_SYS_MDAGM ? 1 : 0};
    const BlasShape sh = c.shape();
    const size_t bb64 = spinor_block_bytes(h->g, SpinorFmt::F64, nrhs);
    void *b64, *x64, *bfull = nullptr;
    COLA_TRY(vec(c, "b64", SpinorFmt::F64, &b64));
    COLA_TRY(vec(c, "x64", SpinorFmt::F64, &x64));
    const bool clover = h->csw != 0.0;

    if (p->system == COLA_SYS_MDAGM) {
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, b64, b, nrhs, -1, st));
    } else if (p->system == COLA_SYS_SCHUR) {
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, b64, b, nrhs, 0, st));
    } else {
        // b_hat_e = b_e + kappa D_eo A_oo^-1 b_o ; rhs = S^H b_hat_e
        COLA_TRY(get_vec(h, "prop_b_full_" + std::to_string(nrhs), 2 * bb64, &bfull));
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, bfull, b, nrhs, -1, st));
        void *to, *bhat;
        COLA_TRY(get_vec(h, "prop_to_" + std::to_string(nrhs), bb64, &to));
        COLA_TRY(get_vec(h, "prop_bhat_" + std::to_string(nrhs), bb64, &bhat));
        const void *bo = (const char *)bfull + bb64;
        if (clover) {
            COLA_HIP(h, launch_clover_site(blas_shape(h->g, nrhs, 1), SpinorFmt::F64, 1, to, bo,
                                           h->clovinv64, 1, st));
        } else {
            COLA_HIP(h, hipMemcpyAsync(to, bo, bb64, hipMemcpyDeviceToDevice, st));
        }
        HopCall hc{bhat, to, 0, 0};
        hc.epi = EPI_XPAY;
        hc.x = bfull;
        hc.a = h->kappa;
        COLA_TRY(hop(h, hc, COLA_FP64, nrhs, st));
        COLA_TRY(apply_op(h, b64, bhat, COLA_OP_SCHUR_DAG, 0, COLA_FP64, nrhs, st));
    }
    if (p->use_x0) {
        COLA_HIP(h, hipMemsetAsync(x64, 0, c.bytes(SpinorFmt::F64), st));
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, x64, x, nrhs, c.full ? -1 : 0, st));
    } else {
        COLA_HIP(h, hipMemsetAsync(x64, 0, c.bytes(SpinorFmt::F64), st));
    }
    // thresholds tol^2 |b_q|^2
    std::vector<double> bn(nrhs), thr(nrhs);
    const Reduce red_b = reduce_into(h, BNORM);
    COLA_HIP(h, launch_norm2(sh, SpinorFmt::F64, b64, red_b, st));
    COLA_TRY(read_slot(c, BNORM, bn.data()));
    for (int q = 0; q < nrhs; ++q) thr[q] = p->tol * p->tol * bn[q];

    Outcome o;
    cola_cg_params_t pp = *p;
    auto run = [&]() -> int {
        o.final_tr.clear();
        switch (pp.scheme) {
            case COLA_CG_FP64: return solve_reliable(c, COLA_FP64, pp, x64, b64, thr, &o);
            case COLA_CG_FP32_RELIABLE: return solve_reliable(c, COLA_FP32, pp, x64, b64, thr, &o);
            case COLA_CG_FP16_DEFECT: return solve_defect(c, COLA_FP16, pp, x64, b64, thr, &o);
            case COLA_CG_FP32_DEFECT: return solve_defect(c, COLA_FP32, pp, x64, b64, thr, &o);
            default: return set_error(h, COLA_EINVAL, "unknown solver scheme");
        }
    };
    // final FP64 true residual of the solved system (the solver's last one when it
    // computed it for the returned x)
    std::vector<double> tr(nrhs);
    auto system_residual = [&]() -> int {
        if ((int)o.final_tr.size() == nrhs) {
            tr = o.final_tr;
        } else {
            void *r64;
            COLA_TRY(vec(c, "r64", SpinorFmt::F64, &r64));
            COLA_TRY(true_residual(c, r64, b64, x64, TRUE_RES));
            COLA_TRY(read_slot(c, TRUE_RES, tr.data()));
        }
        for (int q = 0; q < nrhs; ++q)
            if (!(tr[q] <= thr[q]) && o.status == COLA_OK) o.status = COLA_NOT_CONVERGED;
        return COLA_OK;
    };
    COLA_TRY(run());
    COLA_TRY(system_residual());

    if (p->system == COLA_SYS_PROPAGATOR) {
        // x_o = A_oo^-1 (b_o + kappa D_oe x_e) and the residual of M x = b on the full
        // lattice, one parity block at a time in the solver's FP64 residual block:
        // t = A_pp x_p - kappa D x_{1-p}, then t = b_p - t.  With x_o reconstructed
        // exactly, b - M x is (b_hat - S x_e) on the even sites and zero on the odd ones,
        // which the normal equations bound only up to the condition of S: a column whose
        // full residual misses tol has its normal-system threshold cut by
        // (tol / residual / 2)^2 and the solve continues from x (at most three times).
        void *xfull, *t;
        COLA_TRY(get_vec(h, "prop_x_full_" + std::to_string(nrhs), 2 * bb64, &xfull));
        COLA_TRY(vec(c, "r64", SpinorFmt::F64, &t));
        std::vector<double> bf(nrhs);
        const BlasShape sh1 = blas_shape(h->g, nrhs, 1);
        const BlasShape shf = blas_shape(h->g, nrhs, 2);
        const Reduce red_bf = reduce_into(h, BNORM);
        COLA_HIP(h, launch_norm2(shf, SpinorFmt::F64, bfull, red_bf, st));
        COLA_TRY(read_slot(c, BNORM, bf.data()));
        auto full_residual = [&]() -> int {
            COLA_HIP(h, hipMemcpyAsync(xfull, x64, bb64, hipMemcpyDeviceToDevice, st));
            HopCall hc{(char *)xfull + bb64, x64, 1, 0};
            hc.epi = clover ? EPI_XPAY_CLOV : EPI_XPAY;
            hc.x = (const char *)bfull + bb64;
            hc.a = h->kappa;
            hc.clov = h->clovinv64;
            COLA_TRY(hop(h, hc, COLA_FP64, nrhs, st));
            for (int q = 0; q < 2; ++q) {
                HopCall hm{t, (const char *)xfull + (1 - q) * bb64, q, 0};
                hm.epi = clover ? EPI_CLOV_XPAY : EPI_XPAY;
                hm.x = (const char *)xfull + q * bb64;
                hm.a = -h->kappa;
                hm.clov = h->clov64;
                COLA_TRY(hop(h, hm, COLA_FP64, nrhs, st));
                COLA_HIP(h, launch_residual(sh1, t, (const char *)bfull + q * bb64, t,
                                            reduce_into(h, q == 0 ? TRUE_RES : TMP), st));
            }
            COLA_HIP(h, launch_scalar_add(c.slot(TRUE_RES), c.slot(TMP), nrhs, st));
            return read_slot(c, TRUE_RES, tr.data());
        };
        COLA_TRY(full_residual());
        for (int round = 0; round < 3 && o.status == COLA_OK; ++round) {
            bool again = false;
            for (int q = 0; q < nrhs; ++q) {
                const double lim = p->tol * p->tol * bf[q];
                if (tr[q] > lim) {
                    thr[q] *= 0.25 * lim / tr[q];
                    again = true;
                }
            }
            if (!again) break;
            pp.use_x0 = 1;
            COLA_TRY(run());
            COLA_TRY(system_residual());
            COLA_TRY(full_residual());
        }
        for (int q = 0; q < nrhs; ++q)
            if (!(tr[q] <= p->tol * p->tol * bf[q]) && o.status == COLA_OK)
                o.status = COLA_NOT_CONVERGED;
        bn = bf;
        COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, x, xfull, nrhs, -1, st));
    } else if (p->system == COLA_SYS_SCHUR) {
        COLA_HIP(h, hipMemsetAsync(x, 0, (size_t)h->g.Vh * 2 * 12 * 16 * nrhs, st));
        COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, x, x64, nrhs, 0, st));
    } else {
        COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, x, x64, nrhs, -1, st));
    }
    COLA_HIP(h, hipStreamSynchronize(st));
    if (r) {
        r->status = o.status;
        r->iterations = o.iterations;
        r->outer_cycles = o.outer;
        r->reliable_updates = o.reliable;
        if (r->true_rel_residual)
            for (int q = 0; q < nrhs; ++q)
                r->true_rel_residual[q] = bn[q] > 0 ? std::sqrt(tr[q] / bn[q]) : 0.0;
        r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return o.status;
}

// ---------------------------------------------------------------- multi-shift CG

// (A + sigma_q) x_q = b for nshift shifts sigma_q >= 0 from the Krylov space of the
// unshifted CG on A (M^H M or S^H S, FP64, one rhs).  The shifted residuals stay
// collinear with the base residual, r_q = zeta_q r, and with the base CG's alpha, beta
//   zeta_q' = zeta_q zeta_q^old alpha^old /
//             (alpha beta^old (zeta_q^old - zeta_q) + zeta_q^old alpha^old (1 + sigma_q alpha))
//   x_q += alpha zeta_q'/zeta_q p_q ;  p_q = zeta_q' r' + beta (zeta_q'/zeta_q)^2 p_q
// (zeta = zeta^old = 1, alpha^old = 1, beta^old = 0, p_q = b at the start).  The
// shifts' x and p live as the rhs of one packed field; the scalar recursion runs on
// the host from the base alpha and beta read back each iteration.  A shift stops once
// zeta_q^2 |r|^2 <= tol^2 |b|^2; its true residual is then checked against twice that.
int cg_multishift_impl(cola_handle_t *h, void *x, const void *b, int nshift, const double *sigma,
                       const cola_cg_params_t *p, cola_cg_result_t *res, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    const int full = p->system == COLA_SYS_MDAGM ? 1 : 0;
    Ctx c{h, st, 1, full};
    Ctx cn{h, st, nshift, full};
    const BlasShape sh1 = c.shape(), shn = cn.shape();
    void *b64, *r64, *p64, *ap, *xb, *xs, *ps, *axs;
    COLA_TRY(vec(c, "b64", SpinorFmt::F64, &b64));
    COLA_TRY(vec(c, "r64", SpinorFmt::F64, &r64));
    COLA_TRY(vec(c, "ms_p", SpinorFmt::F64, &p64));
    COLA_TRY(vec(c, "ms_ap", SpinorFmt::F64, &ap));
    COLA_TRY(vec(c, "ms_xb", SpinorFmt::F64, &xb));
    COLA_TRY(vec(cn, "ms_xs", SpinorFmt::F64, &xs));
    COLA_TRY(vec(cn, "ms_ps", SpinorFmt::F64, &ps));
    COLA_TRY(vec(cn, "ms_axs", SpinorFmt::F64, &axs));
    COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, b64, b, 1, full ? -1 : 0, st));
    const size_t b1 = c.bytes(SpinorFmt::F64), bn_ = cn.bytes(SpinorFmt::F64);
    COLA_HIP(h, hipMemcpyAsync(r64, b64, b1, hipMemcpyDeviceToDevice, st));
    COLA_HIP(h, hipMemcpyAsync(p64, b64, b1, hipMemcpyDeviceToDevice, st));
    COLA_HIP(h, hipMemsetAsync(xb, 0, b1, st));
    COLA_HIP(h, hipMemsetAsync(xs, 0, bn_, st));
    COLA_HIP(h, hipMemsetAsync(ps, 0, bn_, st));
    // the shift recursion lives on the device (MsState): init writes the first update's
    // coefficients (p_q = b); each iteration's advance kernel reads the base CG's rho'
    // and pi where the reductions left them.  The host only reads the state's flags at
    // the convergence checks.
    void *state_v;
    COLA_TRY(get_vec(h, "ms_state", sizeof(MsState), &state_v));
    MsState *state = (MsState *)state_v;
    COLA_HIP(h, launch_norm2(sh1, SpinorFmt::F64, b64, reduce_into(h, BNORM), st));
    COLA_HIP(h, launch_ms_init(state, sigma, nshift, p->tol * p->tol, c.slot(BNORM), st));
    COLA_HIP(h, launch_ms_update(shn, xs, ps, r64, &state->coef, st));
    double bnorm = 0.0;
    COLA_TRY(read_slot(c, BNORM, &bnorm));
    COLA_HIP(h, hipMemcpyAsync(c.slot(RHO), c.slot(BNORM), sizeof(double),
                               hipMemcpyDeviceToDevice, st));
    if (full) COLA_TRY(zero_pi2(c));
    COLA_TRY(write_active(c, std::vector<int>{1}));
    const double thr = p->tol * p->tol * bnorm;
    const int check = p->check_interval > 0 ? p->check_interval : default_check(c, 8);
    int status = COLA_OK, it = 0, iters = 0;
    // flags read back from the state: finished, status, iterations (consecutive ints)
    static_assert(offsetof(MsState, status) + sizeof(int) == offsetof(MsState, finished) &&
                      offsetof(MsState, finished) + sizeof(int) == offsetof(MsState, iterations),
                  "state flag order");
    bool finished = bnorm == 0.0;
    int flags[3] = {COLA_OK, finished ? 1 : 0, 0};
    while (!finished) {
        if (it >= p->max_iter) {
            status = COLA_NOT_CONVERGED;
            break;
        }
        COLA_TRY(normal(c, COLA_FP64, ap, p64));
        COLA_HIP(h, launch_cg_xr(sh1, SpinorFmt::F64, SpinorFmt::F64, SpinorFmt::F64,
                                 SpinorFmt::F64, xb, p64, r64, ap, c.slot(RHO), c.slot(PI),
                                 full ? c.slot(PI2) : nullptr, h->active,
                                 reduce_into(h, RHO_NEW), st));
        COLA_HIP(h, launch_ms_advance(state, c.slot(RHO_NEW), c.slot(PI),
                                      full ? c.slot(PI2) : nullptr, st));
        COLA_HIP(h, launch_ms_update(shn, xs, ps, r64, &state->coef, st));
        COLA_HIP(h, launch_cg_p(sh1, SpinorFmt::F64, SpinorFmt::F64, r64, p64, c.slot(RHO_NEW),
                                c.slot(RHO), h->active, st));
        COLA_TRY(rotate_rho(c));
        ++it;
        if (it % check == 0 || it >= p->max_iter) {
            COLA_HIP(h, hipMemcpyAsync(flags, &state->status, sizeof flags,
                                       hipMemcpyDeviceToHost, st));
            COLA_HIP(h, hipStreamSynchronize(st));
            // flags: status, finished, iterations
            if (flags[0] != COLA_OK) {
                status = flags[0];
                break;
            }
            finished = flags[1] != 0;
        }
    }
    iters = finished ? flags[2] : it;
    // true residuals |b - (A + sigma_q) x_q| / |b|, all shifts in one multi-rhs pass
    std::vector<double> tr(nshift, 0.0);
    COLA_TRY(normal(cn, COLA_FP64, axs, xs));
    COLA_HIP(h, launch_ms_residual(shn, b64, axs, xs, sigma, reduce_into(h, TRUE_RES), st));
    COLA_TRY(read_slot(cn, TRUE_RES, tr.data()));
    // the recursive residuals drift from the true ones by rounding: a shift counts as
    // converged within twice the tolerance
    for (int q = 0; q < nshift; ++q)
        if (!(tr[q] <= 4.0 * thr) && status == COLA_OK) status = COLA_NOT_CONVERGED;
    if (!full) COLA_HIP(h, hipMemsetAsync(x, 0, (size_t)h->g.Vh * 2 * 12 * 16 * nshift, st));
    COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, x, xs, nshift, full ? -1 : 0, st));
    COLA_HIP(h, hipStreamSynchronize(st));
    if (res) {
        res->status = status;
        res->iterations = iters;
        res->outer_cycles = 0;
        res->reliable_updates = 0;
        if (res->true_rel_residual)
            for (int q = 0; q < nshift; ++q)
                res->true_rel_residual[q] = bnorm > 0 ? std::sqrt(tr[q] / bnorm) : 0.0;
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace cola
