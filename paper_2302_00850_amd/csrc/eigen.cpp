// Low-eigenmode solver and deflated CG (host side).
//
// The paper lists solvers for eigenmodes beside the linear-system solvers among COLA's
// key algorithms, after Kalkreuter and Simma's accelerated conjugate-gradient method.
// That method finds the n lowest eigenpairs of the Hermitian positive normal operator
// A (M^H M on the full lattice or S^H S on the even sites) by minimising Rayleigh
// quotients one vector at a time, each kept orthogonal to the vectors before it:
//
//   sweep: for i = 0 .. n-1
//     x = x_i with its components along x_0 .. x_{i-1} removed, normalised; y = A x;
//     CG on the unit sphere: gradient g = P (y - mu x) with mu = <x, y> and P the
//     projector off x_0 .. x_{i-1}; direction p = g + (|g|^2 / |g_old|^2) p; the
//     exact line search takes the lower eigenvector (u0, u1) of A restricted to
//     {x, q} (q the normalised part of P p orthogonal to x, z = A q):
//       x = u0 x + u1 q, y = u0 y + u1 z (renormalised);
//     stop once |g| has fallen by inner_reduction (the acceleration) or after
//     inner_max steps;
//   Rayleigh-Ritz: H = X^H A X, H = W diag(lambda) W^H, X = X W, eigenvalues
//   ascending; repeat until every |A x_i - lambda_i x_i| <= tol lambda_i.
//
// One application of A per CG step, in FP64 through the operator kernels; the vector
// algebra runs in the eig_dots / eig_lincomb kernels; the scalars (2 x 2 and n x n
// Hermitian eigenproblems, line-search coefficients) on the host.
//
// Deflated CG: the starting guess is the low-mode part of the solution,
// x0 = sum_i x_i <x_i, b> / lambda_i, then the chosen CG scheme continues from it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "handle.h"
#include "small_eig.h"

namespace cola {

int cg_solve_impl(cola_handle_t *h, void *x, const void *b, int nrhs, const cola_cg_params_t *p,
                  cola_cg_result_t *r, hipStream_t st);

namespace {

struct Eig {
    cola_handle_t *h;
    hipStream_t st;
    int full;      // 1: M^H M on both parity blocks, 0: S^H S on the even block
    size_t n;      // complex entries per packed vector (padding sites stay zero)
    size_t bytes;  // bytes per packed vector
    double *dres;  // device results of the dot launches (2 kEigMax doubles)
};

int alloc(const Eig &e, const std::string &tag, void **out) {
    return get_vec(e.h, "eig_" + tag + "_" + std::to_string(e.full), e.bytes, out);
}

// <V_j, w> into device result slots off + j (no wait)
int dots_at(const Eig &e, const std::vector<const void *> &V, const void *w, size_t off) {
    const size_t m = V.size();
    for (size_t j0 = 0; j0 < m; j0 += kEigChunk) {
        const int k = (int)std::min<size_t>(kEigChunk, m - j0);
        EigVecs vv{};
        for (int j = 0; j < k; ++j) vv.v[j] = (const Cplx64 *)V[j0 + j];
        COLA_HIP(e.h, launch_eig_dots(vv, k, w, e.n, e.h->partial, e.dres + 2 * (off + j0),
                                      e.st));
    }
    return COLA_OK;
}

// the first m result slots, after the queued launches (one wait)
int read_dots(const Eig &e, size_t m, std::vector<cd> &out) {
    out.assign(m, cd(0, 0));
    if (m == 0) return COLA_OK;
    COLA_HIP(e.h, hipMemcpyAsync(e.h->host_scal, e.dres, sizeof(double) * 2 * m,
                                 hipMemcpyDeviceToHost, e.st));
    COLA_HIP(e.h, hipStreamSynchronize(e.st));
    for (size_t j = 0; j < m; ++j) out[j] = cd(e.h->host_scal[2 * j], e.h->host_scal[2 * j + 1]);
    return COLA_OK;
}

// out[j] = <V_j, w>
int dots(const Eig &e, const std::vector<const void *> &V, const void *w, std::vector<cd> &out) {
    COLA_TRY(dots_at(e, V, w, 0));
    return read_dots(e, V.size(), out);
}

// out = a out + sum_j c_j V_j (a = 0: out is overwritten)
int lincomb(const Eig &e, void *out, cd a, const std::vector<const void *> &V,
            const std::vector<cd> &c) {
    const size_t m = V.size();
    size_t j0 = 0;
    do {
        const int k = (int)std::min<size_t>(kEigChunk, m - j0);
        EigVecs vv{};
        EigCoef cc{};
        for (int j = 0; j < k; ++j) {
            vv.v[j] = (const Cplx64 *)V[j0 + j];
            cc.c[j] = {c[j0 + j].real(), c[j0 + j].imag()};
        }
        const cd aa = j0 == 0 ? a : cd(1, 0);
        COLA_HIP(e.h, launch_eig_lincomb(out, aa.real(), aa.imag(), vv, cc, k, e.n, e.st));
        j0 += (size_t)k;
    } while (j0 < m);
    return COLA_OK;
}

// out = a out + sum_j c_j V_j, and |out|^2 into result slot 0 (no wait)
int lincomb_norm(const Eig &e, void *out, cd a, const std::vector<const void *> &V,
                 const std::vector<cd> &c) {
    const size_t m = V.size();
    size_t j0 = 0;
    do {
        const int k = (int)std::min<size_t>(kEigChunk, m - j0);
        EigVecs vv{};
        EigCoef cc{};
        for (int j = 0; j < k; ++j) {
            vv.v[j] = (const Cplx64 *)V[j0 + j];
            cc.c[j] = {c[j0 + j].real(), c[j0 + j].imag()};
        }
        const cd aa = j0 == 0 ? a : cd(1, 0);
        const bool last = j0 + (size_t)k >= m;
        COLA_HIP(e.h, launch_eig_lincomb(out, aa.real(), aa.imag(), vv, cc, k, e.n, e.st,
                                         last ? e.h->partial : nullptr,
                                         last ? e.dres : nullptr));
        j0 += (size_t)k;
    } while (j0 < m);
    return COLA_OK;
}

int copy(const Eig &e, void *dst, const void *src) {
    COLA_HIP(e.h, hipMemcpyAsync(dst, src, e.bytes, hipMemcpyDeviceToDevice, e.st));
    return COLA_OK;
}

int norm(const Eig &e, const void *v, double *out) {
    std::vector<cd> d;
    COLA_TRY(dots(e, {v}, v, d));
    *out = std::sqrt(std::max(0.0, d[0].real()));
    return COLA_OK;
}

int apply_A(const Eig &e, void *out, const void *in) {
    return apply_op(e.h, out, in, e.full ? COLA_OP_MDAGM : COLA_OP_SCHUR_DAGSCHUR, 0, COLA_FP64,
                    1, e.st);
}

// v -= sum_{j < i} X_j <X_j, v>
int project(const Eig &e, const std::vector<void *> &X, int i, void *v) {
    if (i == 0) return COLA_OK;
    std::vector<const void *> V(X.begin(), X.begin() + i);
    std::vector<cd> d;
    COLA_TRY(dots(e, V, v, d));
    for (auto &z : d) z = -z;
    return lincomb(e, v, cd(1, 0), V, d);
}

}  // namespace

int eigensolve_impl(cola_handle_t *h, void *Xc, int nv, const cola_eig_params_t *p,
                    cola_eig_result_t *res, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    const int full = p->system == COLA_SYS_MDAGM ? 1 : 0;
    const size_t bb = spinor_block_bytes(h->g, SpinorFmt::F64, 1);
    Eig e{h, st, full, (size_t)12 * h->g.S * (full ? 2 : 1), bb * (full ? 2 : 1), nullptr};
    void *dres;
    COLA_TRY(get_vec(h, "eig_dres", sizeof(double) * 2 * kEigMax, &dres));
    e.dres = (double *)dres;
    const int parity = full ? -1 : 0;
    const size_t canon = (size_t)h->g.Vh * 2 * 12 * 16;  // bytes of one canonical spinor
    int napply = 0, sweeps = 0, status = COLA_NOT_CONVERGED;
    // a breakdown leaves X as it came and reports the status in *res as well
    auto breakdown = [&](const char *msg) {
        if (res) {
            res->status = COLA_BREAKDOWN;
            res->sweeps = sweeps;
            res->applications = napply;
            res->seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return set_error(h, COLA_BREAKDOWN, msg);
    };

    std::vector<void *> X(nv), Y(nv), T(nv);
    for (int i = 0; i < nv; ++i) {
        COLA_TRY(alloc(e, "X" + std::to_string(i), &X[i]));
        COLA_TRY(alloc(e, "Y" + std::to_string(i), &Y[i]));
        COLA_TRY(alloc(e, "T" + std::to_string(i), &T[i]));
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, X[i], (const char *)Xc + i * canon,
                                       1, parity, st));
    }
    void *q, *z, *g, *pv, *tmp;
    COLA_TRY(alloc(e, "q", &q));
    COLA_TRY(alloc(e, "z", &z));
    COLA_TRY(alloc(e, "g", &g));
    COLA_TRY(alloc(e, "p", &pv));
    COLA_TRY(alloc(e, "tmp", &tmp));

    const double red = p->inner_reduction > 0 ? p->inner_reduction : 0.1;
    const int inner_max = p->inner_max > 0 ? p->inner_max : 50;
    const int max_sweeps = p->max_sweeps > 0 ? p->max_sweeps : 100;
    std::vector<double> lam(nv, 0.0), resid(nv, 0.0);
    std::vector<cd> d;

    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        sweeps = sweep;
        for (int i = 0; i < nv; ++i) {
            void *x = X[i], *y = Y[i];
            double nx, n0;
            COLA_TRY(norm(e, x, &n0));
            COLA_TRY(project(e, X, i, x));
            COLA_TRY(norm(e, x, &nx));
            // nothing left after removing the earlier vectors (beyond rounding): x_i lies
            // in their span
            if (!(nx > 1e-10 * n0) || !std::isfinite(nx))
                return breakdown("starting vectors are linearly dependent or not finite");
            COLA_TRY(lincomb(e, x, cd(1 / nx, 0), {}, {}));
            COLA_TRY(apply_A(e, y, x));
            ++napply;
            COLA_TRY(dots(e, {x}, y, d));
            double mu = d[0].real();
            COLA_TRY(lincomb(e, g, cd(0, 0), {y, x}, {cd(1, 0), cd(-mu, 0)}));
            COLA_TRY(project(e, X, i, g));
            COLA_TRY(dots(e, {g}, g, d));
            double gn2 = d[0].real();
            const double g0 = std::sqrt(std::max(0.0, gn2));
            COLA_TRY(copy(e, pv, g));
            // Host waits per step: five (the two projections, the products with z, the
            // renormalisation, |g|^2).  Projecting q off X_0..X_{i-1} and x in one pass
            // equals doing it one after the other, x being orthogonal to the X_j; q and z
            // are used unnormalised, with |q| taken from the same wait as <x, z>, <q, z>;
            // the line-search update, the renormalisation and the gradient run as fused
            // passes (eig_rotate, eig_scale_grad), |g|^2 in the projection's pass.
            std::vector<const void *> Vx(X.begin(), X.begin() + i);
            Vx.push_back(x);
            // q = pv less its components along Vx, formed in one pass from pv
            std::vector<const void *> Vq(Vx);
            Vq.insert(Vq.begin(), pv);
            for (int it = 0; it < inner_max; ++it) {
                if (!(gn2 > 0.0)) break;
                COLA_TRY(dots(e, Vx, pv, d));
                for (auto &c : d) c = -c;
                d.insert(d.begin(), cd(1, 0));
                COLA_TRY(lincomb(e, q, cd(0, 0), Vq, d));
                COLA_TRY(apply_A(e, z, q));
                ++napply;
                COLA_TRY(dots_at(e, {x, q}, z, 0));
                COLA_TRY(dots_at(e, {q}, q, 2));
                COLA_TRY(read_dots(e, 3, d));
                const double qn = std::sqrt(std::max(0.0, d[2].real()));
                if (!(qn > 0.0)) break;
                // with q^ = q / |q|, z^ = z / |q|: <x, z^> = d0 / |q|, <q^, z^> = d1 / |q|^2
                cd u0, u1;
                lower_eigvec(mu, d[0] / qn, d[1].real() / (qn * qn), &u0, &u1);
                // x = u0 x + u1 q^, y = u0 y + u1 z^, with |x|^2 and <x, y> in the same pass
                const cd cq = u1 / qn;
                COLA_HIP(h, launch_eig_rotate(x, y, q, z, {u0.real(), u0.imag()},
                                              {cq.real(), cq.imag()}, e.n, h->partial, e.dres,
                                              st));
                COLA_TRY(read_dots(e, 2, d));
                nx = std::sqrt(std::max(0.0, d[0].real()));
                mu = d[1].real() / (nx * nx);
                // renormalise x, y and form the gradient g = y - mu x in one pass
                COLA_HIP(h, launch_eig_scale_grad(x, y, g, 1 / nx, mu, e.n, st));
                // g off X_0..X_{i-1}, |g|^2 from the same pass
                std::vector<const void *> Vi(X.begin(), X.begin() + i);
                if (i > 0) {
                    COLA_TRY(dots(e, Vi, g, d));
                    for (auto &c : d) c = -c;
                } else {
                    d.clear();
                }
                COLA_TRY(lincomb_norm(e, g, cd(1, 0), Vi, d));
                COLA_TRY(read_dots(e, 1, d));
                const double gnew2 = d[0].real();
                if (!std::isfinite(gnew2))
                    return breakdown("non-finite gradient");
                if (std::sqrt(std::max(0.0, gnew2)) <= red * g0) break;
                COLA_TRY(lincomb(e, pv, cd(gnew2 / gn2, 0), {g}, {cd(1, 0)}));
                gn2 = gnew2;
            }
        }
        // Rayleigh-Ritz on the span of the sweep's vectors
        std::vector<cd> H((size_t)nv * nv);
        std::vector<const void *> Xc_(X.begin(), X.end());
        for (int b = 0; b < nv; ++b) {
            COLA_TRY(dots(e, Xc_, Y[b], d));
            for (int a = 0; a < nv; ++a) H[(size_t)a * nv + b] = d[a];
        }
        for (int a = 0; a < nv; ++a)
            for (int b = a; b < nv; ++b) {
                const cd s = 0.5 * (H[(size_t)a * nv + b] + std::conj(H[(size_t)b * nv + a]));
                H[(size_t)a * nv + b] = s;
                H[(size_t)b * nv + a] = std::conj(s);
            }
        std::vector<cd> W;
        herm_eig(nv, H, lam, W);
        std::vector<cd> col(nv);
        for (int b = 0; b < nv; ++b) {
            for (int a = 0; a < nv; ++a) col[a] = W[(size_t)a * nv + b];
            COLA_TRY(lincomb(e, T[b], cd(0, 0), Xc_, col));
        }
        X.swap(T);
        std::vector<const void *> Yc(Y.begin(), Y.end());
        for (int b = 0; b < nv; ++b) {
            for (int a = 0; a < nv; ++a) col[a] = W[(size_t)a * nv + b];
            COLA_TRY(lincomb(e, T[b], cd(0, 0), Yc, col));
        }
        Y.swap(T);
        bool conv = true;
        for (int i = 0; i < nv; ++i) {
            COLA_TRY(lincomb(e, tmp, cd(0, 0), {Y[i], X[i]}, {cd(1, 0), cd(-lam[i], 0)}));
            double rn;
            COLA_TRY(norm(e, tmp, &rn));
            resid[i] = lam[i] != 0 ? rn / std::fabs(lam[i]) : rn;
            conv &= rn <= p->tol * std::fabs(lam[i]);
        }
        if (conv) {
            status = COLA_OK;
            break;
        }
    }
    // the cache keeps its tags: the vectors now named T belong to X's pool after the
    // swaps, which does not matter, they are all eig work vectors
    for (int i = 0; i < nv; ++i) {
        char *dst = (char *)Xc + i * canon;
        COLA_HIP(h, hipMemsetAsync(dst, 0, canon, st));
        COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, dst, X[i], 1, parity, st));
    }
    COLA_HIP(h, hipStreamSynchronize(st));
    if (res) {
        res->status = status;
        res->sweeps = sweeps;
        res->applications = napply;
        if (res->eigenvalues)
            for (int i = 0; i < nv; ++i) res->eigenvalues[i] = lam[i];
        if (res->residuals)
            for (int i = 0; i < nv; ++i) res->residuals[i] = resid[i];
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int cg_deflated_impl(cola_handle_t *h, void *x, const void *b, int nrhs, const void *Xc,
                     const double *lambda, int nv, const cola_cg_params_t *p,
                     cola_cg_result_t *r, hipStream_t st) {
    const int full = p->system == COLA_SYS_MDAGM ? 1 : 0;
    const size_t bb = spinor_block_bytes(h->g, SpinorFmt::F64, 1);
    Eig e{h, st, full, (size_t)12 * h->g.S * (full ? 2 : 1), bb * (full ? 2 : 1), nullptr};
    void *dres;
    COLA_TRY(get_vec(h, "eig_dres", sizeof(double) * 2 * kEigMax, &dres));
    e.dres = (double *)dres;
    const int parity = full ? -1 : 0;
    const size_t canon = (size_t)h->g.Vh * 2 * 12 * 16;
    std::vector<const void *> X(nv);
    for (int i = 0; i < nv; ++i) {
        void *v;
        COLA_TRY(alloc(e, "D" + std::to_string(i), &v));
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, v, (const char *)Xc + i * canon, 1,
                                       parity, st));
        X[i] = v;
    }
    void *bq, *x0;
    COLA_TRY(alloc(e, "bq", &bq));
    COLA_TRY(alloc(e, "x0", &x0));
    std::vector<cd> d;
    for (int q = 0; q < nrhs; ++q) {
        COLA_HIP(h, launch_pack_spinor(h->g, SpinorFmt::F64, bq, (const char *)b + q * canon, 1,
                                       parity, st));
        COLA_TRY(dots(e, X, bq, d));
        for (int i = 0; i < nv; ++i) d[i] /= lambda[i];
        COLA_TRY(lincomb(e, x0, cd(0, 0), X, d));
        char *xq = (char *)x + q * canon;
        COLA_HIP(h, hipMemsetAsync(xq, 0, canon, st));
        COLA_HIP(h, launch_unpack_spinor(h->g, SpinorFmt::F64, xq, x0, 1, parity, st));
    }
    cola_cg_params_t p2 = *p;
    p2.use_x0 = 1;
    return cg_solve_impl(h, x, b, nrhs, &p2, r, st);
}

}  // namespace cola
