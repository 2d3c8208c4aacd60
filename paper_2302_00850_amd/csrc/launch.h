// Host-callable launchers for the HIP kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace cola {

// Reduction target: per-block partials, a last-block ticket (kept at 0 between
// launches) and the per-rhs result array; T = site slots per block.
struct Reduce {
    double *partial;
    unsigned *counter;
    double *result;
};

// --- hop
// result[q] = sum of partial[b][q] over b < nblocks in block order (width columns)
hipError_t launch_reduce_partials(const double *partial, int nblocks, int width, double *result,
                                  hipStream_t st);
hipError_t launch_hop(const HopArgs &a, LinkFmt lf, int rpt, int grid, int block, hipStream_t st);

// --- packing
// canonical complex128 U -> every non-null packed format; maxdev receives the
// largest SU(3) deviation (max |U U^H - 1|, |det U - 1|) as the bits of a double.
hipError_t launch_pack_gauge(const Geom &g, const void *U, void *g64_18, void *g64_12,
                             void *g32_12, void *g16_12, unsigned long long *maxdev,
                             hipStream_t st);
// canonical complex128 [nrhs][V][4][3] <-> packed; parity -1 = both parity blocks
hipError_t launch_pack_spinor(const Geom &g, SpinorFmt f, void *dst, const void *src, int nrhs,
                              int parity, hipStream_t st);
hipError_t launch_unpack_spinor(const Geom &g, SpinorFmt f, void *dst, const void *src, int nrhs,
                                int parity, hipStream_t st);

// --- BLAS on packed blocks; nblk = 1 (one parity block) or 2 (full field)
struct BlasShape {
    int S, R, nblk;
    int T;  // site slots per block; threads per block = T * R
    int grid;
};
BlasShape blas_shape(const Geom &g, int nrhs, int nblk);

// Multi-shift CG, FP64, shifts as the rhs of the x and p fields (R = sh.R) and the
// shared residual r a one-rhs field: for active shifts q,
//   x_q += alpha_q p_q ;  p_q = zeta_q r + beta_q p_q
struct MsCoef {
    double alpha[kRedMaxWidth], zeta[kRedMaxWidth], beta[kRedMaxWidth];
    int active[kRedMaxWidth];
};
// The shift recursion's state in device memory: a one-thread kernel advances it each
// iteration from the base CG's rho', pi (+ pi2) and writes the coefficients the update
// kernel reads, so an iteration needs no host round trip.
struct MsState {
    double zeta[kRedMaxWidth], zold[kRedMaxWidth], sigma[kRedMaxWidth];
    double alpha_old, beta_old, rho, thr;
    int done[kRedMaxWidth];
    int nshift;
    int status;      // COLA_OK or COLA_BREAKDOWN (non-finite recursion)
    int finished;    // every shift done
    int iterations;  // iterations advanced while not finished
    MsCoef coef;     // this iteration's x_q, p_q coefficients
};
// state from sigma[nshift], tol^2 and |b|^2 (a device scalar); coef = the first update
// (p_q = b)
hipError_t launch_ms_init(MsState *state, const double *sigma, int nshift, double tol2,
                          const double *bnorm, hipStream_t st);
// one iteration of the recursion from the base rho' and pi (pi2 null: one block)
hipError_t launch_ms_advance(MsState *state, const double *rho_new, const double *pi,
                             const double *pi2, hipStream_t st);
hipError_t launch_ms_update(const BlasShape &sh, void *x, void *p, const void *r,
                            const MsCoef *k, hipStream_t st);
// result_q = |b - ax_q - sigma_q x_q|^2 (b a one-rhs field, ax and x with R = sh.R)
hipError_t launch_ms_residual(const BlasShape &sh, const void *b, const void *ax, const void *x,
                              const double *sigma, const Reduce &red, hipStream_t st);
// a[i] += b[i] for i < n <= 64 (per-rhs scalars)
hipError_t launch_scalar_add(double *a, const double *b, int n, hipStream_t st);
// a[i] = b[i] for i < n <= 64
hipError_t launch_scalar_copy(double *a, const double *b, int n, hipStream_t st);
// x += alpha p, r -= alpha Ap, result = |r|^2 ;
// alpha_q = active_q ? rho_q / (pi_q + pi2_q) : 0   (pi2 may be null)
hipError_t launch_cg_xr(const BlasShape &b, SpinorFmt fx, SpinorFmt fp, SpinorFmt fr,
                        SpinorFmt fap, void *x, const void *p, void *r, const void *ap,
                        const double *rho, const double *pi, const double *pi2,
                        const int *active, const Reduce &red, hipStream_t st);
// p = r + beta p ; beta_q = active_q ? rho_new_q / rho_q : 0
hipError_t launch_cg_p(const BlasShape &b, SpinorFmt fr, SpinorFmt fp, const void *r, void *p,
                       const double *rho_new, const double *rho, const int *active,
                       hipStream_t st);
// result = |v|^2 per rhs
hipError_t launch_norm2(const BlasShape &b, SpinorFmt f, const void *v, const Reduce &red,
                        hipStream_t st);
// dst = s_q * src (s = NULL: 1; inv_scale: s_q -> 1/s_q), optional |dst|^2
hipError_t launch_convert(const BlasShape &b, SpinorFmt fd, SpinorFmt fs, void *dst,
                          const void *src, const double *s, int inv_scale, const Reduce *red,
                          hipStream_t st);
// dst(FP64) += s_q * src; zero_src: src = 0 afterwards
hipError_t launch_accum(const BlasShape &b, SpinorFmt fs, void *dst, void *src, const double *s,
                        int zero_src, hipStream_t st);
// r = b - ax (all FP64), result = |r|^2
hipError_t launch_residual(const BlasShape &b, void *r, const void *bb, const void *ax,
                           const Reduce &red, hipStream_t st);
// out = C in on the sites of parity `parity` (one block), C = clover blocks
hipError_t launch_clover_site(const BlasShape &b, SpinorFmt f, int clov_double, void *out,
                              const void *in, const void *clov, int parity, hipStream_t st);

// --- block CG on n <= 16 rhs of one packed block (stride S; ncu: compute units of the
// device, for the resident grid of the grid-stride kernels)
// red.result receives G transposed: (b * n + a) * 2 + {re, im} = sum conj(A_a) B_b
hipError_t launch_gram(int S, int n, int ncu, SpinorFmt fa, SpinorFmt fb, const void *A,
                       const void *B, const Reduce &red, hipStream_t st);
// X_b += sum_a P_a alpha_ab, R_b -= sum_a Q_a alpha_ab (alpha row-major complex FP64);
// with gram, also the Gram matrix R^H R of the updated R into gram->result (as launch_gram)
hipError_t launch_block_axpy(int S, int n, int ncu, SpinorFmt fx, SpinorFmt fp, void *X,
                             const void *P, void *R, const void *Q, const double *alpha,
                             const Reduce *gram, hipStream_t st);
// Z = H^-1 B over the active columns (bit mask act), H and B Gram results (transposed
// layout), pivots below 1e-13 of the largest diagonal deflated; Z row-major (one thread)
hipError_t launch_block_solve(const double *H, const double *B, unsigned act, int n, double *Z,
                              hipStream_t st);
// Pn_b = R_b + sum_a P_a beta_ab
hipError_t launch_block_xpay(int S, int n, int ncu, SpinorFmt fr, SpinorFmt fp, void *Pn,
                             const void *R, const void *P, const double *beta, hipStream_t st);

// --- low-eigenmode solver: one-rhs FP64 packed fields as flat arrays of n complex values
constexpr int kEigChunk = 8;        // vectors per dot / linear-combination launch
constexpr int kEigMaxBlocks = 2048; // blocks of a dot launch (partials: 2 kEigChunk each)
struct EigVecs {
    const Cplx64 *v[kEigChunk];
};
struct EigCoef {
    Cplx64 c[kEigChunk];
};
// result[2j], result[2j+1] = Re, Im <V_j, w> for j < k <= kEigChunk (partial: handle buffer)
hipError_t launch_eig_dots(const EigVecs &V, int k, const void *w, size_t n, double *partial,
                           double *result, hipStream_t st);
// out = a out + sum_{j<k} c_j V_j (a = 0: out is not read; out may be one of the V_j);
// with result non-null also result[0] = |out|^2, result[1] = 0 (after the update)
hipError_t launch_eig_lincomb(void *out, double are, double aim, const EigVecs &V,
                              const EigCoef &c, int k, size_t n, hipStream_t st,
                              double *partial = nullptr, double *result = nullptr);
// x = u x + c q, y = u y + c z (u, c complex), then result[0] = |x|^2, result[1] = 0,
// result[2], result[3] = Re, Im <x, y>
hipError_t launch_eig_rotate(void *x, void *y, const void *q, const void *z, Cplx64 u, Cplx64 c,
                             size_t n, double *partial, double *result, hipStream_t st);
// x *= s, y *= s, g = y - mu x (s, mu real)
hipError_t launch_eig_scale_grad(void *x, void *y, void *g, double s, double mu, size_t n,
                                 hipStream_t st);

// --- clover
// Builds A = 1 - kappa csw sum sigma F (two 6x6 chiral blocks) and A^-1 per site from
// the canonical FP64 links; writes FP64 and FP32 packed copies.  bad counts sites
// whose blocks were not positive definite.
hipError_t launch_clover_build(const Geom &g, const void *U, double kappa, double csw,
                               void *a64, void *ainv64, void *a32, void *ainv32, int *bad,
                               hipStream_t st);

// --- force
hipError_t launch_force(const Geom &g, const void *gauge64_18, const void *X, const void *Y,
                        void *F, double kappa, const Cplx64 phase[4], int mode, hipStream_t st);

// --- HMC (canonical FP64 fields; one lane per link)
// F = traceless Hermitian force of the Wilson plaquette action with coupling beta
hipError_t launch_gauge_force(const Geom &g, const void *U, void *F, double beta, hipStream_t st);
// P -= eps (F1 + F2) over nlinks 3x3 matrices (F2 may be null)
hipError_t launch_momentum_update(void *P, const void *F1, const void *F2, double eps,
                                  size_t nlinks, hipStream_t st);
// U <- exp(i eps P) U over nlinks links, rows re-orthonormalised (row 2 = conj(row0 x row1))
hipError_t launch_link_update(void *U, const void *P, double eps, size_t nlinks, hipStream_t st);
// one APE smearing sweep Out = P_SU3[(1 - alpha) U + alpha/6 staples] (Out != U)
hipError_t launch_ape_sweep(const Geom &g, const void *U, void *Out, double alpha,
                            hipStream_t st);
// *result (device) = sum over sites and mu < nu of Re Tr U_plaq
hipError_t launch_plaquette_sum(const Geom &g, const void *U, double *partial, double *result,
                                hipStream_t st);
// *result = sum |a_k|^2 over n complex entries
hipError_t launch_sqnorm(const void *a, size_t n, double *partial, double *result,
                         hipStream_t st);
// *result = Re sum conj(a_k) b_k over n complex entries
hipError_t launch_redot(const void *a, const void *b, size_t n, double *partial, double *result,
                        hipStream_t st);

}  // namespace cola
