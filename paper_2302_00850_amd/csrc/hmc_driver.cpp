// HMC entry points and the leapfrog trajectory driver (hybrid Monte Carlo, the gauge-field
// generation algorithm in the paper's list, after Duane et al.).  The driver sequences
// the library's own kernels: gauge force, fermion solve and force (the FP64 CG on
// M^H M, Y = M X, the link-wise force kernel), momentum and link updates, and the
// reductions that give H.
#include <chrono>
#include <cmath>
#include <string>

#include "cola.h"
#include "handle.h"
#include "launch.h"

using namespace cola;

namespace {

hipStream_t hstream(void *s) { return (hipStream_t)s; }

size_t nlinks(const cola_handle_t *h) { return (size_t)8 * h->g.Vh; }

// device scratch of the trajectory: forces, fermion vectors, packed M X, scalars
struct HmcWork {
    void *Fg = nullptr, *Ff = nullptr;  // gauge / fermion force (canonical gauge shape)
    void *X = nullptr, *Y = nullptr;    // canonical spinors
    void *Xp = nullptr, *Yp = nullptr;  // packed FP64 full-lattice spinors
    double *sc = nullptr;               // 4 device scalars
};

int scalars(cola_handle_t *h, double **sc) {
    void *p;
    COLA_TRY(get_vec(h, "hmc_sc", 4 * sizeof(double), &p));
    *sc = (double *)p;
    return COLA_OK;
}

int work(cola_handle_t *h, bool fermions, HmcWork *w) {
    const size_t gb = nlinks(h) * 9 * 16;
    COLA_TRY(get_vec(h, "hmc_Fg", gb, &w->Fg));
    COLA_TRY(scalars(h, &w->sc));
    if (!fermions) return COLA_OK;
    const size_t sb = (size_t)2 * h->g.Vh * 12 * 16;
    const size_t pb = cola_field_bytes(h, COLA_FP64, 1, -1);
    COLA_TRY(get_vec(h, "hmc_Ff", gb, &w->Ff));
    COLA_TRY(get_vec(h, "hmc_X", sb, &w->X));
    COLA_TRY(get_vec(h, "hmc_Y", sb, &w->Y));
    COLA_TRY(get_vec(h, "hmc_Xp", pb, &w->Xp));
    COLA_TRY(get_vec(h, "hmc_Yp", pb, &w->Yp));
    return COLA_OK;
}

double read_scalar(cola_handle_t *h, const double *d, hipStream_t st, int *rc) {
    double v = 0.0;
    hipError_t e = hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) *rc = hip_error(h, e, "hmc scalar read-back");
    return v;
}

// Even-odd pseudofermion S_f = phi_e^H (S^H S)^{-1} phi_e (plain Wilson): with
// X_e = (S^H S)^{-1} phi_e and Y_e = S X_e,
//   dS_f = 2 kappa^2 Re[Y_e^H dD_eo X_o + Y_o^H dD_oe X_e],  X_o = D_oe X_e, Y_o = D_eo^H Y_e,
// which is the full-lattice fermion force of (X_e, X_o) and (Y_e, Y_o) with kappa^2 in
// place of kappa.  The handle's gauge field is already packed from U.
int forces_eo(cola_handle_t *h, const void *phi, const cola_hmc_params_t *p, HmcWork &w,
              bool first, bool energy, double *sf, int *iters, int *status, hipStream_t st) {
    cola_cg_params_t cp{};
    cp.system = COLA_SYS_SCHUR;
    cp.scheme = p->cg_scheme;
    cp.tol = p->cg_tol;
    cp.max_iter = p->cg_max_iter;
    cp.reliable_interval = 50;
    cp.use_x0 = first ? 0 : 1;
    double res = 0.0;
    cola_cg_result_t cr{};
    cr.true_rel_residual = &res;
    COLA_TRY(cola_cg_solve(h, w.X, phi, 1, &cp, &cr, st));  // odd sites of X set to 0
    *iters += cr.iterations;
    if (cr.status != COLA_OK) *status = COLA_NOT_CONVERGED;
    const size_t blk = cola_field_bytes(h, COLA_FP64, 1, 0);
    char *xe = (char *)w.Xp, *xo = xe + blk, *ye = (char *)w.Yp, *yo = ye + blk;
    COLA_TRY(cola_pack_spinor(h, w.Xp, w.X, COLA_FP64, 1, -1, st));
    COLA_TRY(cola_dslash_apply(h, xo, xe, COLA_OP_HOP, 1, COLA_FP64, 1, st));
    COLA_TRY(cola_dslash_apply(h, ye, xe, COLA_OP_SCHUR, 0, COLA_FP64, 1, st));
    COLA_TRY(cola_dslash_apply(h, yo, ye, COLA_OP_HOP_DAG, 1, COLA_FP64, 1, st));
    COLA_TRY(cola_unpack_spinor(h, w.Y, w.Yp, COLA_FP64, 1, -1, st));
    if (energy) {
        // X still has zero odd sites here: Re <phi, X> = Re <phi_e, X_e>
        COLA_HIP(h, launch_redot(phi, w.X, (size_t)2 * h->g.Vh * 12, h->partial, w.sc + 1, st));
        int rc = COLA_OK;
        *sf = read_scalar(h, w.sc + 1, st, &rc);
        COLA_TRY(rc);
    }
    COLA_TRY(cola_unpack_spinor(h, w.X, w.Xp, COLA_FP64, 1, -1, st));
    COLA_HIP(h, launch_force(h->g, h->gauge[0], w.X, w.Y, w.Ff, h->kappa * h->kappa, h->phase,
                             COLA_FORCE_LIE, st));
    return COLA_OK;
}

// Forces at the current U into w.Fg (and w.Ff with fermions); with `energy`, the parts
// of H that depend on U: *sg = S_g, *sf = S_f = Re <phi, X>.  X of the previous call is
// the CG's starting guess.
int forces(cola_handle_t *h, void *U, const void *phi, const cola_hmc_params_t *p, HmcWork &w,
           bool first, bool energy, double *sg, double *sf, int *iters, int *status,
           hipStream_t st) {
    COLA_HIP(h, launch_gauge_force(h->g, U, w.Fg, p->beta, st));
    if (energy) {
        COLA_HIP(h, launch_plaquette_sum(h->g, U, h->partial, w.sc, st));
        int rc = COLA_OK;
        const double plaq = read_scalar(h, w.sc, st, &rc);
        COLA_TRY(rc);
        *sg = p->beta * (6.0 * 2.0 * h->g.Vh - plaq / 3.0);
    }
    if (!phi) {
        if (energy) *sf = 0.0;
        return COLA_OK;
    }
    COLA_TRY(cola_set_gauge(h, U, st));
    if (p->eo) return forces_eo(h, phi, p, w, first, energy, sf, iters, status, st);
    cola_cg_params_t cp{};
    cp.system = COLA_SYS_MDAGM;
    cp.scheme = p->cg_scheme;
    cp.tol = p->cg_tol;
    cp.max_iter = p->cg_max_iter;
    cp.reliable_interval = 50;
    cp.use_x0 = first ? 0 : 1;
    double res = 0.0;
    cola_cg_result_t cr{};
    cr.true_rel_residual = &res;
    COLA_TRY(cola_cg_solve(h, w.X, phi, 1, &cp, &cr, st));
    *iters += cr.iterations;
    if (cr.status != COLA_OK) *status = COLA_NOT_CONVERGED;
    // Y = M X through the packed FP64 field
    COLA_TRY(cola_pack_spinor(h, w.Xp, w.X, COLA_FP64, 1, -1, st));
    COLA_TRY(cola_dslash_apply(h, w.Yp, w.Xp, COLA_OP_M, -1, COLA_FP64, 1, st));
    COLA_TRY(cola_unpack_spinor(h, w.Y, w.Yp, COLA_FP64, 1, -1, st));
    COLA_TRY(cola_fermion_force(h, w.Ff, w.X, w.Y, COLA_FORCE_LIE, st));
    if (energy) {
        COLA_HIP(h, launch_redot(phi, w.X, (size_t)2 * h->g.Vh * 12, h->partial, w.sc + 1, st));
        int rc = COLA_OK;
        *sf = read_scalar(h, w.sc + 1, st, &rc);
        COLA_TRY(rc);
    }
    return COLA_OK;
}

int kinetic(cola_handle_t *h, const void *P, HmcWork &w, hipStream_t st, double *k) {
    COLA_HIP(h, launch_sqnorm(P, nlinks(h) * 9, h->partial, w.sc + 2, st));
    int rc = COLA_OK;
    *k = 0.5 * read_scalar(h, w.sc + 2, st, &rc);
    return rc;
}

}  // namespace

int cola_gauge_force(cola_handle_t *h, void *F, const void *U, double beta, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!F || !U) return set_error(h, COLA_EINVAL, "null pointer");
    COLA_HIP(h, launch_gauge_force(h->g, U, F, beta, hstream(stream)));
    return COLA_OK;
}

int cola_fermion_action(cola_handle_t *h, const void *phi, void *X, void *Y, double tol,
                        double *S, int *iterations, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!phi || !X || !Y || !S) return set_error(h, COLA_EINVAL, "null pointer");
    if (!(tol > 0.0) || !std::isfinite(tol)) return set_error(h, COLA_EINVAL, "need tol > 0");
    if (h->csw != 0.0)
        return set_error(h, COLA_EINVAL, "the action's force exists for plain Wilson only");
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    hipStream_t st = hstream(stream);
    void *Xp, *Yp;
    double *sc;
    const size_t pb = cola_field_bytes(h, COLA_FP64, 1, -1);
    COLA_TRY(get_vec(h, "fa_Xp", pb, &Xp));
    COLA_TRY(get_vec(h, "fa_Yp", pb, &Yp));
    COLA_TRY(scalars(h, &sc));
    // X = (M^H M)^{-1} phi from x = 0
    cola_cg_params_t cp{};
    cp.system = COLA_SYS_MDAGM;
    cp.scheme = COLA_CG_FP64;
    cp.tol = tol;
    cp.max_iter = 100000;
    cp.reliable_interval = 50;
    double res = 0.0;
    cola_cg_result_t cr{};
    cr.true_rel_residual = &res;
    COLA_TRY(cola_cg_solve(h, X, phi, 1, &cp, &cr, st));
    if (iterations) *iterations = cr.iterations;
    // Y = M X through the packed FP64 field; S = Re <phi, X>
    COLA_TRY(cola_pack_spinor(h, Xp, X, COLA_FP64, 1, -1, st));
    COLA_TRY(cola_dslash_apply(h, Yp, Xp, COLA_OP_M, -1, COLA_FP64, 1, st));
    COLA_TRY(cola_unpack_spinor(h, Y, Yp, COLA_FP64, 1, -1, st));
    COLA_HIP(h, launch_redot(phi, X, (size_t)2 * h->g.Vh * 12, h->partial, sc + 3, st));
    int rc = COLA_OK;
    *S = read_scalar(h, sc + 3, st, &rc);
    COLA_TRY(rc);
    return cr.status == COLA_OK ? COLA_OK : cr.status;
}

int cola_gauge_action(cola_handle_t *h, const void *U, double beta, double *S, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!U || !S) return set_error(h, COLA_EINVAL, "null pointer");
    double *sc;
    COLA_TRY(scalars(h, &sc));
    hipStream_t st = hstream(stream);
    COLA_HIP(h, launch_plaquette_sum(h->g, U, h->partial, sc, st));
    int rc = COLA_OK;
    const double plaq = read_scalar(h, sc, st, &rc);
    COLA_TRY(rc);
    *S = beta * (6.0 * 2.0 * h->g.Vh - plaq / 3.0);
    return COLA_OK;
}

int cola_link_update(cola_handle_t *h, void *U, const void *P, double eps, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!U || !P) return set_error(h, COLA_EINVAL, "null pointer");
    if (!std::isfinite(eps)) return set_error(h, COLA_EINVAL, "non-finite step");
    COLA_HIP(h, launch_link_update(U, P, eps, nlinks(h), hstream(stream)));
    return COLA_OK;
}

int cola_momentum_update(cola_handle_t *h, void *P, const void *F1, const void *F2, double eps,
                         void *stream) {
    if (!h) return COLA_EINVAL;
    if (!P || !F1) return set_error(h, COLA_EINVAL, "null pointer");
    COLA_HIP(h, launch_momentum_update(P, F1, F2, eps, nlinks(h), hstream(stream)));
    return COLA_OK;
}

int cola_hmc_trajectory(cola_handle_t *h, void *U, void *P, const void *phi,
                        const cola_hmc_params_t *p, cola_hmc_result_t *r, void *stream) {
    if (!h) return COLA_EINVAL;
    if (!U || !P || !p || !r) return set_error(h, COLA_EINVAL, "null pointer");
    if (p->nsteps < 1 || !(p->eps > 0.0) || !std::isfinite(p->eps) || !std::isfinite(p->beta))
        return set_error(h, COLA_EINVAL, "need nsteps >= 1, finite eps > 0 and finite beta");
    if (phi && h->csw != 0.0)
        return set_error(h, COLA_EINVAL, "fermion force of the clover term not available");
    if (h->flic)
        return set_error(h, COLA_EINVAL,
                         "the trajectory driver runs the Wilson operator (the FLIC force, "
                         "through the smearing, is not built)");
    if (phi && (!(p->cg_tol > 0.0) || p->cg_max_iter < 1))
        return set_error(h, COLA_EINVAL, "need cg_tol > 0 and cg_max_iter >= 1");
    if (phi && (p->cg_scheme < COLA_CG_FP64 || p->cg_scheme > COLA_CG_FP32_DEFECT))
        return set_error(h, COLA_EINVAL, "unknown cg_scheme");
    if (p->integrator < 0 || p->integrator > 2)
        return set_error(h, COLA_EINVAL,
                         "integrator must be 0 (leapfrog), 1 (Omelyan) or 2 (two time scales)");
    if (p->integrator == 2 && p->n_gauge < 1)
        return set_error(h, COLA_EINVAL, "n_gauge must be >= 1");
    hipStream_t st = hstream(stream);
    const auto t0 = std::chrono::steady_clock::now();
    HmcWork w;
    COLA_TRY(work(h, phi != nullptr, &w));
    *r = cola_hmc_result_t{};
    r->status = COLA_OK;
    const size_t nl = nlinks(h);
    const double eps = p->eps;
    int status = COLA_OK, iters = 0;

    // H0 and the force at the start
    COLA_TRY(kinetic(h, P, w, st, &r->kinetic0));
    COLA_TRY(forces(h, U, phi, p, w, true, true, &r->gauge0, &r->fermion0, &iters, &status, st));
    const void *Ff = phi ? w.Ff : nullptr;
    if (p->integrator == 0) {
        // leapfrog: P eps/2, then per step U eps and P eps (eps/2 after the last)
        COLA_HIP(h, launch_momentum_update(P, w.Fg, Ff, 0.5 * eps, nl, st));
        for (int k = 0; k < p->nsteps; ++k) {
            COLA_HIP(h, launch_link_update(U, P, eps, nl, st));
            const bool last = k == p->nsteps - 1;
            COLA_TRY(forces(h, U, phi, p, w, false, last, &r->gauge1, &r->fermion1, &iters,
                            &status, st));
            COLA_HIP(h, launch_momentum_update(P, w.Fg, Ff, last ? 0.5 * eps : eps, nl, st));
        }
    } else if (p->integrator == 2) {
        // two time scales: fermion kicks of eps around n_gauge gauge leapfrog sub-steps of
        // eps / n_gauge (w.Fg and w.Ff hold the forces at the current U)
        const int m = p->n_gauge;
        const double hs = eps / m;
        if (Ff) COLA_HIP(h, launch_momentum_update(P, Ff, nullptr, 0.5 * eps, nl, st));
        for (int k = 0; k < p->nsteps; ++k) {
            const bool last = k == p->nsteps - 1;
            COLA_HIP(h, launch_momentum_update(P, w.Fg, nullptr, 0.5 * hs, nl, st));
            for (int j = 0; j < m; ++j) {
                COLA_HIP(h, launch_link_update(U, P, hs, nl, st));
                COLA_HIP(h, launch_gauge_force(h->g, U, w.Fg, p->beta, st));
                COLA_HIP(h, launch_momentum_update(P, w.Fg, nullptr, j < m - 1 ? hs : 0.5 * hs,
                                                   nl, st));
            }
            // the fermion force (and, after the last step, the energies) at the new U
            COLA_TRY(forces(h, U, phi, p, w, false, last, &r->gauge1, &r->fermion1, &iters,
                            &status, st));
            if (Ff)
                COLA_HIP(h, launch_momentum_update(P, Ff, nullptr, last ? 0.5 * eps : eps, nl,
                                                   st));
        }
    } else {
        // Omelyan: P lambda eps, then per step U eps/2, P (1 - 2 lambda) eps, U eps/2 and
        // P 2 lambda eps (the next step's first momentum step merged; lambda eps after the
        // last)
        const double lam = 0.1931833275037836;
        COLA_HIP(h, launch_momentum_update(P, w.Fg, Ff, lam * eps, nl, st));
        for (int k = 0; k < p->nsteps; ++k) {
            const bool last = k == p->nsteps - 1;
            COLA_HIP(h, launch_link_update(U, P, 0.5 * eps, nl, st));
            COLA_TRY(forces(h, U, phi, p, w, false, false, nullptr, nullptr, &iters, &status,
                            st));
            COLA_HIP(h, launch_momentum_update(P, w.Fg, Ff, (1.0 - 2.0 * lam) * eps, nl, st));
            COLA_HIP(h, launch_link_update(U, P, 0.5 * eps, nl, st));
            COLA_TRY(forces(h, U, phi, p, w, false, last, &r->gauge1, &r->fermion1, &iters,
                            &status, st));
            COLA_HIP(h, launch_momentum_update(P, w.Fg, Ff, (last ? lam : 2.0 * lam) * eps, nl,
                                               st));
        }
    }
    COLA_TRY(kinetic(h, P, w, st, &r->kinetic1));
    COLA_HIP(h, hipStreamSynchronize(st));
    r->H0 = r->kinetic0 + r->gauge0 + r->fermion0;
    r->H1 = r->kinetic1 + r->gauge1 + r->fermion1;
    r->dH = r->H1 - r->H0;
    r->cg_iterations = iters;
    r->status = status;
    r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return COLA_OK;
}
