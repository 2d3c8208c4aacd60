/*
 * cola.h -- C ABI of the MI355X (gfx950) Wilson-Dirac library.
 *
 * The library implements the data-parallel hot path of the CG fermion-matrix
 * inverter that the paper (Kamleh, "Evolving the COLA software library",
 * Lattice 2022) describes: the Wilson(-clover) Dirac operator applied to a
 * fermion field ("fermion matrix"), conjugate-gradient solves with it in
 * plain FP64 and in mixed precision (32-bit inner iterations, 64-bit outer
 * solver), and the force term of Hybrid Monte Carlo; around them, the HMC
 * molecular-dynamics trajectory (gauge force, link and momentum updates, leapfrog and
 * Omelyan integrators) and the multi-shift CG of rational HMC.  The paper's GPU code is
 * reached from Fortran through an ISO C binding; this header is the same kind
 * of plain-C boundary: POD types, raw pointers, no C++ or torch types.
 *
 * Conventions (all entry points):
 *   lattice   dims = {Lx, Ly, Lz, Lt}, all even and >= 2; mu = 0,1,2,3 = x,y,z,t;
 *             site = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) mod 2.
 *   operator  (M psi)(x) = A(x) psi(x) - kappa sum_mu [ (1-g_mu) e+_mu(x) U_mu(x) psi(x+mu)
 *                                                   + (1+g_mu) e-_mu(x) U_mu(x-mu)^H psi(x-mu) ]
 *             chiral (DeGrand-Rossi) gammas; e+_mu(x) = bc_phase[mu] when x_mu = L_mu-1,
 *             e-_mu(x) = conj(bc_phase[mu]) when x_mu = 0, else 1; A = 1 (csw = 0) or the
 *             clover matrix 1 - kappa*csw*sum_{mu<nu} sigma_mu,nu F_mu,nu (csw != 0).
 *             M^H = g5 M g5.
 *   canonical complex128 (re, im interleaved) device arrays, row-major:
 *             gauge  U[Lt][Lz][Ly][Lx][mu][row][col]
 *             spinor psi[nrhs][Lt][Lz][Ly][Lx][spin][colour]
 *   packed    the library's own per-parity structure-of-arrays form in one of the
 *             precisions below (see cola_field_bytes); made by cola_pack_spinor.
 *   streams   `stream` is a hipStream_t (NULL = default stream).  dslash_apply,
 *             pack/unpack, the forces and the link/momentum updates are asynchronous on
 *             it; set_gauge, the solvers, gauge_action and hmc_trajectory synchronise it
 *             before returning.
 *   ownership the caller owns every buffer passed in; the library owns its packed
 *             gauge/clover copies and its workspace, released by cola_destroy.
 *   errors    0 = COLA_OK; negative = nothing valid was produced (message in
 *             cola_last_error); positive = output valid but flagged.
 *   threads   a handle is not re-entrant: one handle per host thread / stream.
 */
#ifndef COLA_H
#define COLA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COLA_ABI_VERSION 2

/* status codes */
enum {
    COLA_OK = 0,
    COLA_EINVAL = -1,       /* bad argument, unsupported combination, bad dims      */
    COLA_EHIP = -2,         /* a HIP runtime call failed (text in cola_last_error)  */
    COLA_ENOMEM = -3,       /* device allocation failed                             */
    COLA_ESTATE = -4,       /* call out of order (e.g. no gauge field set)          */
    COLA_NOT_CONVERGED = 1, /* cg: max_iter reached; x holds the last iterate       */
    COLA_BREAKDOWN = 2      /* cg: NaN/Inf or a vanishing denominator               */
};

/* storage precision of packed fields: spinor format / link format */
enum {
    COLA_FP64 = 0,    /* FP64 spinors, FP64 links with all 18 reals               */
    COLA_FP64_12 = 1, /* FP64 spinors, FP64 links, rows 0-1 stored (12 reals)     */
    COLA_FP32 = 2,    /* FP32 spinors, FP32 links, 12 reals, FP32 arithmetic      */
    COLA_FP16 = 3     /* FP16 spinors + one FP32 scale per site and rhs, FP16 links
                         (12 reals), FP32 arithmetic                                */
};

/* operators for cola_dslash_apply */
enum {
    COLA_OP_HOP = 0,            /* out_p = D_{p,1-p} in_{1-p}  (half lattice, parity p)  */
    COLA_OP_HOP_DAG = 1,        /* out_p = (D^H)_{p,1-p} in_{1-p}                        */
    COLA_OP_M = 2,              /* full lattice M                                        */
    COLA_OP_MDAG = 3,           /* full lattice M^H                                      */
    COLA_OP_MDAGM = 4,          /* full lattice M^H M                                    */
    COLA_OP_SCHUR = 5,          /* even sites: S = A_ee - kappa^2 D_eo A_oo^-1 D_oe      */
    COLA_OP_SCHUR_DAG = 6,      /* S^H                                                   */
    COLA_OP_SCHUR_DAGSCHUR = 7  /* S^H S                                                 */
};

/* linear systems for cola_cg_solve */
enum {
    COLA_SYS_MDAGM = 0,      /* M^H M x = b on the full lattice                         */
    COLA_SYS_SCHUR = 1,      /* S^H S x_e = b_e on even sites (odd sites of x set to 0) */
    COLA_SYS_PROPAGATOR = 2  /* M x = b, through S^H S on even sites + odd reconstruction */
};

/* solver schemes */
enum {
    COLA_CG_FP64 = 0,          /* plain FP64 CG                                        */
    COLA_CG_FP32_RELIABLE = 1, /* FP32 CG, FP64 x accumulator, FP64 true residual every
                                  reliable_interval iterations and at convergence       */
    COLA_CG_FP16_DEFECT = 2,   /* FP64 defect correction around an FP16-storage inner CG */
    COLA_CG_FP32_DEFECT = 3    /* FP64 defect correction around an FP32 inner CG         */
};

/* cola_create flags */
enum {
    COLA_FLAG_TIMING = 1u /* bracket every hop launch with HIP events (cola_get_stats) */
};

/* force modes */
enum {
    COLA_FORCE_GRAD = 0, /* G = dS/dRe U + i dS/dIm U                                  */
    COLA_FORCE_LIE = 1   /* traceless Hermitian F with dS/de = Tr(H F), U -> e^{ieH} U  */
};

typedef struct cola_handle cola_handle_t;

typedef struct {
    int system;            /* COLA_SYS_*                                                */
    int scheme;            /* COLA_CG_*                                                 */
    int block;             /* 0: independent CG per column, batched (lockstep);
                              1: O'Leary block CG sharing one Krylov space, as the inner
                              solver of the DEFECT schemes on the SCHUR and PROPAGATOR
                              systems (COLA_EINVAL otherwise)                          */
    double tol;            /* stop when ||b - A x|| / ||b|| <= tol for every column,
                              A the system's operator (M for PROPAGATOR, whose normal
                              equations are tightened per column until the full-lattice
                              residual meets tol), checked in FP64                      */
    int max_iter;          /* cap on (inner) iterations, summed over outer cycles       */
    int reliable_interval; /* FP32_RELIABLE: iterations between FP64 residual updates   */
    double inner_tol;      /* DEFECT: relative residual reduction of each inner solve
                              (0: 1e-2 for FP16, 1e-5 for FP32)                         */
    int use_x0;            /* 1: x holds the initial guess on entry                     */
    int check_interval;    /* iterations between host convergence checks; 0: every
                              iteration when one iteration applies the operator to at
                              least 2^20 site-rhs (the host wait is then negligible),
                              else 8 (5 for FP32_RELIABLE)                              */
} cola_cg_params_t;

typedef struct {
    int status;                /* COLA_OK, COLA_NOT_CONVERGED or COLA_BREAKDOWN         */
    int iterations;            /* total (inner) CG iterations                          */
    int outer_cycles;          /* defect-correction cycles                             */
    int reliable_updates;      /* FP64 residual recomputations inside the solve         */
    double *true_rel_residual; /* caller-owned host array[nrhs] (may be NULL): final
                                  FP64 ||b - A x|| / ||b|| per column                   */
    double seconds;            /* wall time of the solve                                */
} cola_cg_result_t;

typedef struct {
    int system;             /* COLA_SYS_MDAGM (A = M^H M) or COLA_SYS_SCHUR (A = S^H S on
                               the even sites)                                          */
    double tol;             /* stop when |A x_i - lambda_i x_i| <= tol lambda_i for all i */
    double inner_reduction; /* gradient reduction that ends one vector's minimisation in
                               a sweep (the acceleration; 0: 0.1)                       */
    int inner_max;          /* CG steps per vector and sweep at most (0: 50)            */
    int max_sweeps;         /* sweeps at most (0: 100)                                  */
} cola_eig_params_t;

typedef struct {
    int status;          /* COLA_OK or COLA_NOT_CONVERGED (max_sweeps reached)          */
    int sweeps;          /* sweeps done                                                 */
    int applications;    /* applications of A                                           */
    double *eigenvalues; /* caller-owned host array[n] (may be NULL): ascending        */
    double *residuals;   /* caller-owned host array[n] (may be NULL):
                            |A x_i - lambda_i x_i| / lambda_i                           */
    double seconds;      /* wall time                                                   */
} cola_eig_result_t;

/* Kinds of hop launch (the epilogue fused into the half-lattice hop D_{p,1-p}), the second
 * index of the per-kind accounting below.  x: a same-parity spinor, C: clover blocks. */
enum {
    COLA_HOP_PLAIN = 0,        /* out = D in                                             */
    COLA_HOP_XPAY = 1,         /* out = x + a D in                                       */
    COLA_HOP_CLOV = 2,         /* out = C D in                                           */
    COLA_HOP_CLOV_XPAY = 3,    /* out = C x + a D in                                     */
    COLA_HOP_XPAY_CLOV = 4,    /* out = C (x + a D in)                                   */
    COLA_HOP_XPAY_CG = 5,      /* CG update of x and r with x + a D in (nothing stored)  */
    COLA_HOP_CLOV_XPAY_CG = 6, /* CG update of x and r with C x + a D in                 */
    COLA_HOP_KINDS = 8
};

/* Hop-kernel accounting, per storage precision (index COLA_FP64 .. COLA_FP16), filled
 * only for handles created with COLA_FLAG_TIMING.  Algorithmic bytes count every
 * link, input spinor and output spinor of a launch once (plus the epilogue's extra
 * spinor / clover reads); flops count 1320 per site and rhs, 42 per rebuilt link
 * row, 48 per axpy and 552 per clover application. */
typedef struct {
    long long hop_launches[4]; /* hop kernels launched                                */
    double hop_seconds[4];     /* summed HIP-event durations, on the launch stream     */
    double hop_bytes[4];       /* summed algorithmic bytes                             */
    double hop_flops[4];       /* summed flops                                         */
    /* the same per precision and launch kind (COLA_HOP_*) */
    long long kind_launches[4][COLA_HOP_KINDS];
    double kind_seconds[4][COLA_HOP_KINDS];
    double kind_bytes[4][COLA_HOP_KINDS];
} cola_stats_t;

/* ---------------------------------------------------------------- lifecycle */

int cola_abi_version(void);

/* Create a handle on the current HIP device.  dims: {Lx,Ly,Lz,Lt}, all even, >= 2.
 * bc_phase: 8 doubles, (re, im) of e^{i theta_mu} for mu = 0..3 (antiperiodic time:
 * {1,0, 1,0, 1,0, -1,0}).  csw = 0 selects plain Wilson.  Returns COLA_EINVAL for
 * bad dims, a null h or non-finite kappa/csw. */
int cola_create(cola_handle_t **h, const int dims[4], double kappa, const double bc_phase[8],
                double csw, unsigned flags);
int cola_destroy(cola_handle_t *h);
/* Text of the last error on h (empty string if none; never NULL). */
const char *cola_last_error(const cola_handle_t *h);

/* ------------------------------------------------------------------- fields */

/* Copy in the gauge field (canonical complex128 device array) and build every
 * packed form (FP64 18-real; 12-real FP64/FP32/FP16 when every link is SU(3) to
 * 1e-12) plus the clover blocks and their inverses when csw != 0.  Synchronises
 * `stream`.  Compressed precisions are refused later (COLA_EINVAL) if the field
 * is not SU(3).  The canonical array is not retained. */
int cola_set_gauge(cola_handle_t *h, const void *U_dev, void *stream);

/* 1 when the current gauge field passed the SU(3) check (12-real forms usable). */
int cola_gauge_is_su3(const cola_handle_t *h);

/* Bytes of a packed spinor field of precision `prec` with nrhs right-hand sides on
 * one parity (parity 0 or 1) or on the full lattice (parity -1).  0 on bad args. */
size_t cola_field_bytes(const cola_handle_t *h, int prec, int nrhs, int parity);

/* canonical complex128 [nrhs][Lt][Lz][Ly][Lx][4][3] <-> packed.  parity -1 packs the
 * full lattice; parity 0/1 packs only that parity's sites (unpack of one parity
 * leaves the other parity's sites of dst untouched).  FP16 rounds to nearest even
 * after dividing by the per-site, per-rhs max |component|. */
int cola_pack_spinor(cola_handle_t *h, void *dst_packed, const void *src_canon, int prec,
                     int nrhs, int parity, void *stream);
int cola_unpack_spinor(cola_handle_t *h, void *dst_canon, const void *src_packed, int prec,
                       int nrhs, int parity, void *stream);

/* -------------------------------------------------------------- hot path */

/* The fermion matrix applied to a fermion field (the paper's GPU "fermion matrix
 * inverter" is built on it; its remark that lattice codes are memory-bandwidth bound is
 * why the stencil stores 12-real links and FP16/FP32 spinors).
 * out = op(in) on packed fields of precision `prec` with nrhs right-hand sides.
 * HOP/HOP_DAG: in is the parity (1-parity) block, out the `parity` block.
 * M/MDAG/MDAGM: full-lattice fields.  SCHUR*: even-parity blocks (parity ignored).
 * out and in must not overlap.  Asynchronous on `stream`. */
int cola_dslash_apply(cola_handle_t *h, void *out, const void *in, int op, int parity, int prec,
                      int nrhs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cola_dslash_apply with the same
 * arguments, layouts and results (bitwise), which allocates nothing.  The intermediate
 * vectors of the composed operators (M^H M: one full field; S and S^H: one odd block;
 * S^H S: an even and an odd block) live in a fixed device workspace of
 * COLA_NOALLOC_SCRATCH_BYTES (128 MiB) per device, a static array of the library that
 * each device holds until the process ends; its address is taken at cola_create.
 * Returns COLA_EINVAL (with a message naming both sizes) when the operator needs more
 * workspace than that, before touching any buffer.  The hops run in the cached or the
 * default launch shape: no tuning, no timing events (COLA_FLAG_TIMING is ignored).
 * Every call on a device shares that device's workspace: calls that overlap on one
 * device (two streams, two threads, two handles) race, so the caller orders them.
 * Nothing in the workspace has to start at zero (each intermediate is written in full
 * before it is read).  Asynchronous on `stream`. */
#define COLA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int cola_dslash_apply_noalloc(cola_handle_t *h, void *out, const void *in, int op, int parity,
                              int prec, int nrhs, void *stream);

/* Conjugate-gradient solve with the fermion matrix (the paper's linear-system solvers and
 * its GPU CG benchmark: 32-bit inner iterations inside a 64-bit outer solver, after the
 * mixed-precision methods of Clark et al. that it cites).
 * Solve for nrhs right-hand sides; x and b are canonical complex128 device arrays
 * [nrhs][Lt][Lz][Ly][Lx][4][3].  For COLA_SYS_SCHUR only the even sites of b are
 * read and the odd sites of x are set to zero.  Synchronises `stream`.  Returns
 * COLA_OK, COLA_NOT_CONVERGED (x = best iterate) or COLA_BREAKDOWN, or < 0.
 * The CG update of x and r runs inside the last hop of S^dag S (even-odd systems) or
 * the two parity hops of M^dag (full lattice), so A p is never stored; the environment
 * variable COLA_CG_FUSE=0 selects a separate update kernel instead (same iterates up to
 * the order of the |r|^2 sums). */
int cola_cg_solve(cola_handle_t *h, void *x, const void *b, int nrhs, const cola_cg_params_t *p,
                  cola_cg_result_t *r, void *stream);

/* Multi-shift CG (the shifted solves of rational HMC, Kennedy et al. in the paper's
 * list of algorithms): (A + shifts[q]) x_q = b for q < nshift (1 .. 16, shifts >= 0)
 * from one Krylov space, A = M^H M (COLA_SYS_MDAGM) or S^H S on the even sites
 * (COLA_SYS_SCHUR), FP64 only (p->scheme = COLA_CG_FP64, p->block = 0).  b: one canonical
 * complex128 spinor; x: canonical [nshift][Lt][Lz][Ly][Lx][4][3] (SCHUR: odd sites set
 * to zero).  A shift stops when its iterated residual reaches p->tol |b|; status is
 * COLA_NOT_CONVERGED if a true residual exceeds 2 p->tol |b| (the iterated and true
 * residuals differ by rounding).  r->iterations counts the shared iterations,
 * r->true_rel_residual[q] (caller array of nshift) is |b - (A + sigma_q) x_q| / |b|.
 * Returns like cola_cg_solve; COLA_EINVAL for other systems or schemes, nshift out of
 * range or a negative shift.  Synchronises `stream`. */
int cola_cg_multishift(cola_handle_t *h, void *x, const void *b, int nshift, const double *shifts,
                       const cola_cg_params_t *p, cola_cg_result_t *r, void *stream);

/* Low eigenmodes (the paper's eigenmode solvers, after Kalkreuter and Simma's
 * accelerated conjugate-gradient method): the n lowest eigenpairs of A = M^H M or S^H S
 * by minimising the Rayleigh quotient of one vector at a time by CG, each vector kept
 * orthogonal to the ones before it, the minimisation of a vector stopped early once its
 * gradient has fallen by p->inner_reduction, and a Rayleigh-Ritz rotation of the n
 * vectors after each sweep, until every residual meets p->tol.  FP64 throughout.
 * X: canonical complex128 [n][Lt][Lz][Ly][Lx][4][3] device array, the starting vectors
 * on entry (linearly independent; SCHUR reads their even sites) and the orthonormal
 * eigenvectors on return (SCHUR: odd sites zero), ascending eigenvalues in
 * r->eigenvalues.  n = 1 .. 32.  Returns COLA_OK, COLA_NOT_CONVERGED (the current
 * vectors and Ritz values are returned), COLA_BREAKDOWN (a vector with nothing left
 * once the vectors before it are projected out, as a zero start or one in the span of
 * the starts before it that have not moved yet, or non-finite values; X unchanged) or
 * < 0: COLA_EINVAL for another system, n out of
 * range, tol <= 0 or csw-free requirements unmet, COLA_ESTATE without a gauge field.
 * Synchronises `stream`. */
int cola_eigensolve(cola_handle_t *h, void *X, int n, const cola_eig_params_t *p,
                    cola_eig_result_t *r, void *stream);

/* Deflated CG: cola_cg_solve on the MDAGM or SCHUR system started from the low-mode part
 * of the solution, x0 = sum_i X_i <X_i, b> / lambda[i], with n eigenpairs of that
 * system's A (from cola_eigensolve: X canonical complex128 [n][...] device array,
 * lambda a host array).  Any scheme; p->use_x0 is ignored (x is overwritten with x0 on
 * entry).  Returns like cola_cg_solve; COLA_EINVAL for the PROPAGATOR system, n out of
 * 1 .. 32 or a non-positive eigenvalue. */
int cola_cg_deflated(cola_handle_t *h, void *x, const void *b, int nrhs, const void *X,
                     const double *lambda, int n, const cola_cg_params_t *p,
                     cola_cg_result_t *r, void *stream);

/* The HMC fermion force (the paper's gauge-field generation by Hybrid Monte Carlo, after
 * Duane et al., in its list of key algorithms): link-wise outer products of two solve
 * vectors.
 * Fermion force of S = phi^H (M^H M)^{-1} phi for plain Wilson M, from X = (M^H M)^{-1} phi
 * and Y = M X (canonical complex128 spinors, nrhs = 1).  F: canonical gauge-shaped
 * complex128 output [Lt][Lz][Ly][Lx][4][3][3].  COLA_EINVAL when csw != 0 (the clover
 * term's own force is not implemented).  Asynchronous on `stream`. */
int cola_fermion_force(cola_handle_t *h, void *F_dev, const void *X_dev, const void *Y_dev,
                       int mode, void *stream);

/* Pseudofermion action S = phi^H (M^H M)^{-1} phi of plain Wilson M on the handle's gauge
 * field (the action whose derivative the HMC fermion force is; the paper's list of key
 * algorithms, HMC after Duane et al.): X = (M^H M)^{-1} phi by FP64 CG from x = 0 to the
 * FP64 true relative residual tol, Y = M X, and *S = Re <phi, X> (host double) from a
 * deterministic device reduction.  phi, X, Y: canonical complex128 device spinors
 * [Lt][Lz][Ly][Lx][4][3]; X and Y are written (the inputs of cola_fermion_force).
 * *iterations (may be NULL) receives the CG iteration count.  Returns COLA_OK,
 * COLA_NOT_CONVERGED or COLA_BREAKDOWN from the solve (X, Y and S are filled from the last
 * iterate), COLA_EINVAL for null pointers, tol <= 0 or csw != 0, COLA_ESTATE without a
 * gauge field.  Synchronises `stream`. */
int cola_fermion_action(cola_handle_t *h, const void *phi_dev, void *X_dev, void *Y_dev,
                        double tol, double *S, int *iterations, void *stream);

/* ------------------------------------------------ FLIC (fat-link irrelevant clover)
 * The CSSM action family the paper's physics programme uses (the FLIC and fat-link HMC
 * entries of its bibliography): the relevant part of the Wilson-Dirac operator keeps the
 * thin links U, the irrelevant Wilson and clover terms use APE-smeared links F:
 *   M psi = A_F psi - kappa sum_mu [(F_mu(x) - g_mu U_mu(x)) e+ psi(x+mu)
 *                                   + (F_mu(x-mu)^H + g_mu U_mu(x-mu)^H) e- psi(x-mu)]
 * with A_F the clover matrix of F (csw != 0) or 1.  F = U gives the Wilson(-clover)
 * operator. */

/* APE smearing: nsweeps sweeps of V_mu(x) = (1 - alpha) U_mu(x) + (alpha / 6) (sum of the
 * six staples around the link), each projected to the nearest SU(3) matrix (unitary
 * polar factor, determinant phase removed with the principal cube root).  F and U:
 * canonical complex128 [Lt][Lz][Ly][Lx][4][3][3] device arrays (F may be U); periodic
 * links.  nsweeps = 0 copies U.  Asynchronous on `stream`. */
int cola_ape_smear(cola_handle_t *h, void *F, const void *U, double alpha, int nsweeps,
                   void *stream);

/* Switch the handle to the FLIC operator with smeared links F (canonical, SU(3) to 1e-12)
 * and the thin links of the last cola_set_gauge; the clover term (csw != 0) is rebuilt
 * from F.  Every operator, solver and eigensolver call then applies FLIC, in FP64 and
 * FP32 (COLA_FP16 is refused); cola_fermion_force and cola_hmc_trajectory refuse it.
 * cola_set_gauge returns the handle to the Wilson(-clover) operator.  COLA_ESTATE
 * before cola_set_gauge.  Synchronises `stream`. */
int cola_set_fat_gauge(cola_handle_t *h, const void *F, void *stream);

/* -------------------------------------------------------------------- HMC */
/* Hybrid Monte Carlo (the paper's gauge-field generation algorithm, after Duane et al.,
 * in its list of algorithms) for SU(3) links with the Wilson plaquette action
 *   S_g = beta sum_{x, mu<nu} (1 - Re Tr U_mu,nu(x) / 3)
 * plus, when a pseudofermion phi is given, S_f = phi^H (M^H M)^{-1} phi for plain Wilson
 * M (the handle's kappa and boundary phases).  Momenta P are traceless Hermitian per
 * link, H = sum Tr(P^2) / 2 + S_g + S_f, links move as U -> exp(i eps P) U and the
 * forces are in the COLA_FORCE_LIE form.  U, P and F are canonical complex128 device
 * arrays [Lt][Lz][Ly][Lx][4][3][3]; phi a canonical spinor.  All asynchronous on
 * `stream` unless stated. */

/* F = force of S_g (traceless Hermitian, dS_g/de = Tr(H F) along U -> e^{ieH} U). */
int cola_gauge_force(cola_handle_t *h, void *F_dev, const void *U_dev, double beta,
                     void *stream);
/* *S = S_g(U) (host double); synchronises `stream`. */
int cola_gauge_action(cola_handle_t *h, const void *U_dev, double beta, double *S,
                      void *stream);
/* U <- exp(i eps P) U on every link (in place), each link's rows then re-orthonormalised
 * (row 2 = conj(row0 x row1)), so that rounding does not move U off SU(3) over many
 * updates (the compressed link formats require SU(3) to 1e-12). */
int cola_link_update(cola_handle_t *h, void *U_dev, const void *P_dev, double eps, void *stream);
/* P -= eps (F1 + F2) on every link (F2 may be NULL). */
int cola_momentum_update(cola_handle_t *h, void *P_dev, const void *F1_dev, const void *F2_dev,
                         double eps, void *stream);

typedef struct {
    double beta;     /* gauge coupling                                              */
    double eps;      /* molecular-dynamics step size                                */
    int nsteps;      /* integrator steps (trajectory length eps * nsteps)           */
    double cg_tol;   /* FP64 CG tolerance of the fermion solves (phi given)        */
    int cg_max_iter; /* cap per solve                                               */
    int eo;          /* 1: even-odd pseudofermion S_f = phi_e^H (S^H S)^{-1} phi_e,
                        S = 1 - kappa^2 D_eo D_oe, phi's odd sites ignored (its solves
                        run on the half lattice); 0: phi^H (M^H M)^{-1} phi            */
    int integrator;  /* 0: leapfrog (nsteps + 1 force evaluations); 1: second-order
                        minimum-norm (Omelyan, lambda = 0.1931833275037836; 2 nsteps + 1
                        force evaluations, a smaller energy violation per step);
                        2: leapfrog on two time scales, the fermion force on steps of
                        eps and the gauge force on n_gauge sub-steps of eps / n_gauge  */
    int n_gauge;     /* gauge sub-steps per step for integrator 2 (>= 1)               */
    int cg_scheme;   /* COLA_CG_* of the fermion solves (0 = FP64); the mixed schemes
                        still reach cg_tol in FP64 true residual                        */
} cola_hmc_params_t;

typedef struct {
    int status;           /* COLA_OK, or COLA_NOT_CONVERGED if a fermion solve failed */
    double H0, H1;        /* Hamiltonian before and after                             */
    double dH;            /* H1 - H0 (Metropolis: accept with probability min(1, e^-dH)) */
    double kinetic0, kinetic1, gauge0, gauge1, fermion0, fermion1; /* parts of H0, H1   */
    int cg_iterations;    /* summed over all fermion solves of the trajectory         */
    double seconds;       /* wall time                                                */
} cola_hmc_result_t;

/* One trajectory in place on U and P (leapfrog: half step in P, nsteps alternating link
 * and momentum steps, half step in P; or the other integrators above); phi = NULL for
 * the pure gauge theory.  The accept/reject decision is the caller's (it keeps a copy of
 * U and draws the uniform number).  With phi: needs csw = 0, re-packs the handle's gauge
 * field from U before every fermion solve (cola_set_gauge) and leaves it packed from
 * the final U.  Returns COLA_EINVAL for nsteps < 1, eps <= 0, non-finite parameters, an
 * unknown integrator or cg_scheme, or n_gauge < 1 with integrator 2.  Synchronises
 * `stream`. */
int cola_hmc_trajectory(cola_handle_t *h, void *U_dev, void *P_dev, const void *phi_dev,
                        const cola_hmc_params_t *p, cola_hmc_result_t *r, void *stream);

/* ---------------------------------------------------------- diagnostics */

int cola_get_stats(cola_handle_t *h, cola_stats_t *s); /* synchronises pending timings */
int cola_reset_stats(cola_handle_t *h);

/* Autotuning of the hop launch shape (the paper's remark that performance hinges on
 * how lattice sites map to GPU threads, in its paragraph on the GPU execution model):
 * sites per block, rhs per thread, grid (natural or resident), time chunk, spatial tile
 * and LDS staging of the site's links.  Every shape gives bitwise the same result.
 * Keys are (lattice, precision, nrhs, epilogue, fused norm).
 * mode 0: off (defaults), 1: tune on first use of a key (each candidate timed on the
 * caller's buffers, so that first call takes longer), 2: re-tune every key.
 * Tuned shapes go into a per-handle table and into a process-wide table kept in a text
 * file ($COLA_TUNE_CACHE, empty for none; else $XDG_CACHE_HOME/cola/hop_tune.txt or
 * ~/.cache/cola/hop_tune.txt), one line per (device, key).  With tuning off, a hop takes
 * the handle's tuned shape, else the stored one (the file is read on the first hop of the
 * process), else the default: shapes tuned once are used by default afterwards.
 * COLA_HOP_SHAPE (a measurement knob) overrides the stored shapes.
 * cola_tune_dump writes the handle's table as JSON text into buf (returns the length
 * needed, including the terminating NUL). */
int cola_set_tuning(cola_handle_t *h, int mode);
size_t cola_tune_dump(const cola_handle_t *h, char *buf, size_t len);
/* Merge the file at path (NULL: the default file) into the process-wide table, or write
 * that table there (atomically, creating the directory).  Return the number of entries,
 * or COLA_EINVAL when the file cannot be read or written. */
int cola_tune_load(cola_handle_t *h, const char *path);
int cola_tune_save(cola_handle_t *h, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* COLA_H */
