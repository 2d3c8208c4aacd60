/*
 * FP64 CPU oracle for the Wilson(-clover) Dirac operator, its even-odd Schur
 * complement, conjugate gradient on the normal equations and the HMC fermion
 * force.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, table
 * or header with the GPU library: its own gamma table, its own site indexing,
 * plain loops over sites, full 4x4 spin matrices (no spin projection), full
 * 3x3 links (no compression), complex128 throughout.
 *
 * The paper (Kamleh, "Evolving the COLA software library", Lattice 2022)
 * names the algorithms -- linear-system solves with the fermion matrix, mixed
 * 32/64-bit CG, gauge-field generation with HMC -- but prints no formula.  The
 * operator below is the textbook Wilson-Dirac convention:
 *
 *   (M psi)(x) = A(x) psi(x) - kappa * sum_mu [ (1 - g_mu) e+_mu(x) U_mu(x) psi(x+mu)
 *                                             + (1 + g_mu) e-_mu(x) U_mu(x-mu)^H psi(x-mu) ]
 *
 * with e+_mu(x) = exp(i theta_mu) when x_mu = L_mu - 1 (else 1), e-_mu(x) its
 * conjugate when x_mu = 0 (else 1), A = 1 for plain Wilson and the
 * Sheikholeslami-Wohlert clover matrix otherwise.  Chiral (DeGrand-Rossi)
 * gamma basis.  Site index = x + Lx*(y + Ly*(z + Lz*t)); spinor entry
 * (site*4 + spin)*3 + colour; link entry ((site*4 + mu)*3 + row)*3 + col.
 * Parity of a site = (x+y+z+t) mod 2.
 *
 * The clover convention A = 1 - kappa*c_sw*sum_{mu<nu} sigma_mu,nu F_mu,nu is a
 * reading (the paper prints no formula); its overall sign and normalisation are
 * pinned by tree-level O(a) improvement: in a constant abelian field, c_sw = 1
 * cancels the Wilson term's shift of the would-be zero modes.  Every function
 * here is pinned by closed forms, invariants or brute force in the CPU
 * test-suite:
 *   oracle_gamma          Clifford algebra, gamma5 = diag(1,1,-1,-1)
 *                         (tests/test_oracle_operator.py: test_gamma_table_clifford)
 *   oracle_hop, oracle_apply_M
 *                         free-field symbol and eigenvalues, gamma5-hermiticity, gauge and
 *                         translation covariance, dense 2^4 assembly, extent-2 directions
 *                         (tests/test_oracle_operator.py)
 *   oracle_hop_sites      every site equals oracle_hop (tests/test_oracle_pins.py)
 *   oracle_apply_M_sites  its own per-site clover assembly against oracle_apply_M fed
 *                         oracle_clover, every site, csw 0 and 1, both dagger forms
 *                         (tests/test_oracle_pins.py)
 *   oracle_apply_schur    dense Schur complement (test_oracle_operator.py)
 *   oracle_field_strength, oracle_clover
 *                         U = 1, Hermiticity, chiral blocks, covariance, abelian-flux closed
 *                         form, tree-level O(a) cancellation (tests/test_oracle_clover_force.py)
 *   oracle_site_inverse   dense inverses (test_oracle_solver.py, clover propagator)
 *   oracle_cg             dense LU on 2^4 and 2x2x2x4, free-field FFT propagator
 *                         (tests/test_oracle_solver.py)
 *   oracle_force          finite differences of dense solves, Y = eta, S = |eta|^2, covariance
 *                         (tests/test_oracle_clover_force.py)
 *   oracle_plaquette      U = 1, constant abelian flux per plane, gauge invariance, the numpy
 *                         plaquette action of the HMC oracle (tests/test_oracle_pins.py)
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* DeGrand-Rossi chiral basis; mu = 0,1,2,3 = x,y,z,t; gamma5 = g0 g1 g2 g3 = diag(1,1,-1,-1). */
static const cplx GAMMA[4][4][4] = {
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

/* ------------------------------------------------------------------ geometry */

static long volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void site_coords(const int L[4], long s, int x[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long site_of(const int L[4], const int x[4]) {
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

/* neighbour of site s, displaced by `step` (+1 or -1) along mu, periodic in storage */
static long neighbour(const int L[4], long s, int mu, int step) {
    int x[4];
    site_coords(L, s, x);
    x[mu] = (x[mu] + step + L[mu]) % L[mu];
    return site_of(L, x);
}

static int parity_of(const int L[4], long s) {
    int x[4];
    site_coords(L, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static const cplx *link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* --------------------------------------------------------------- the hopping term */

/*
 * out(x) = sum_mu [ (1 + sg g_mu) e+ U_mu(x) in(x+mu) + (1 - sg g_mu) e- U_mu(x-mu)^H in(x-mu) ]
 * with sg = -1 for D and sg = +1 for D^H = g5 D g5 (dagger != 0).
 */
static void hop_site(const int L[4], const double *bc, const cplx *U, const cplx *in, long s,
                     cplx *out, int dagger) {
    const double sg = dagger ? 1.0 : -1.0;
    {
        int x[4];
        site_coords(L, s, x);
        cplx acc[12];
        for (int k = 0; k < 12; ++k) acc[k] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            const cplx phase = bc[2 * mu] + I * bc[2 * mu + 1];
            cplx chi[12];
            /* forward neighbour */
            const long sf = neighbour(L, s, mu, +1);
            const cplx ef = (x[mu] == L[mu] - 1) ? phase : 1.0;
            const cplx *u = link(U, s, mu);
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int b = 0; b < 3; ++b) v += u[a * 3 + b] * in[sf * 12 + sp * 3 + b];
                    chi[sp * 3 + a] = v;
                }
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx g = 0;
                    for (int t = 0; t < 4; ++t) g += GAMMA[mu][sp][t] * chi[t * 3 + a];
                    acc[sp * 3 + a] += ef * (chi[sp * 3 + a] + sg * g);
                }
            /* backward neighbour */
            const long sb = neighbour(L, s, mu, -1);
            const cplx eb = (x[mu] == 0) ? conj(phase) : 1.0;
            const cplx *w = link(U, sb, mu);
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int b = 0; b < 3; ++b) v += conj(w[b * 3 + a]) * in[sb * 12 + sp * 3 + b];
                    chi[sp * 3 + a] = v;
                }
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx g = 0;
                    for (int t = 0; t < 4; ++t) g += GAMMA[mu][sp][t] * chi[t * 3 + a];
                    acc[sp * 3 + a] += eb * (chi[sp * 3 + a] - sg * g);
                }
        }
        for (int k = 0; k < 12; ++k) out[k] = acc[k];
    }
}

static void hop(const int L[4], const double *bc, const cplx *U, const cplx *in, cplx *out,
                int dagger) {
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) hop_site(L, bc, U, in, s, out + s * 12, dagger);
}

/* out(x) = C(x) in(x) for a per-site 12x12 matrix field C (identity if C == NULL) */
static void site_matrix(const int L[4], const cplx *C, const cplx *in, cplx *out) {
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        if (!C) {
            for (int k = 0; k < 12; ++k) out[s * 12 + k] = in[s * 12 + k];
            continue;
        }
        const cplx *c = C + s * 144;
        for (int i = 0; i < 12; ++i) {
            cplx v = 0;
            for (int j = 0; j < 12; ++j) v += c[i * 12 + j] * in[s * 12 + j];
            out[s * 12 + i] = v;
        }
    }
}

/* zero every site whose parity differs from `keep` */
static void mask_parity(const int L[4], cplx *f, int keep) {
    const long V = volume(L);
    for (long s = 0; s < V; ++s)
        if (parity_of(L, s) != keep)
            for (int k = 0; k < 12; ++k) f[s * 12 + k] = 0;
}

void oracle_hop(const int L[4], const double *bc, const double *U, const double *in, double *out,
                int dagger) {
    hop(L, bc, (const cplx *)U, (const cplx *)in, (cplx *)out, dagger);
}

/* the hopping term at a list of sites only: out[k*12 ..] = (D in)(sites[k]) */
void oracle_hop_sites(const int L[4], const double *bc, const double *U, const double *in,
                      const long *sites, long n, double *out, int dagger) {
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k)
        hop_site(L, bc, (const cplx *)U, (const cplx *)in, sites[k], (cplx *)out + k * 12, dagger);
}

/* M psi = A psi - kappa D psi; M^H = A - kappa D^H since A is Hermitian. */
void oracle_apply_M(const int L[4], double kappa, const double *bc, const double *U,
                    const double *A, const double *in, double *out, int dagger) {
    const long n = volume(L) * 12;
    cplx *h = malloc(sizeof(cplx) * n);
    hop(L, bc, (const cplx *)U, (const cplx *)in, h, dagger);
    site_matrix(L, (const cplx *)A, (const cplx *)in, (cplx *)out);
    cplx *o = (cplx *)out;
    for (long k = 0; k < n; ++k) o[k] -= kappa * h[k];
    free(h);
}

/*
 * Even-site Schur complement of M in the even/odd block form
 *   M = [[A_ee, -kappa D_eo], [-kappa D_oe, A_oo]]:
 *   S = A_ee - kappa^2 D_eo A_oo^{-1} D_oe     (dagger: D -> D^H, A unchanged).
 * Arrays are full-lattice; odd sites of `in` are ignored, odd sites of `out` are 0.
 * Ainv holds A^{-1} per site (NULL for plain Wilson).
 */
void oracle_apply_schur(const int L[4], double kappa, const double *bc, const double *U,
                        const double *A, const double *Ainv, const double *in, double *out,
                        int dagger) {
    const long n = volume(L) * 12;
    cplx *pe = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *t2 = malloc(sizeof(cplx) * n);
    memcpy(pe, in, sizeof(cplx) * n);
    mask_parity(L, pe, 0);
    hop(L, bc, (const cplx *)U, pe, t, dagger); /* D_oe p_e lives on odd sites */
    mask_parity(L, t, 1);
    site_matrix(L, (const cplx *)Ainv, t, t2); /* A_oo^{-1} */
    hop(L, bc, (const cplx *)U, t2, t, dagger); /* D_eo (...) lives on even sites */
    site_matrix(L, (const cplx *)A, pe, (cplx *)out);
    cplx *o = (cplx *)out;
    for (long k = 0; k < n; ++k) o[k] -= kappa * kappa * t[k];
    mask_parity(L, o, 0);
    free(pe);
    free(t);
    free(t2);
}

/* ------------------------------------------------------------------- clover */

static void mat3_mul(const cplx *a, const cplx *b, cplx *c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx v = 0;
            for (int k = 0; k < 3; ++k) v += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = v;
        }
}

static void mat3_dag(const cplx *a, cplx *b) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) b[i * 3 + j] = conj(a[j * 3 + i]);
}

/* c = f0 f1 f2 f3 where each factor is a link (dag=0) or its adjoint (dag=1) */
static void path4(const cplx *m[4], const int dag[4], cplx *c) {
    cplx f[4][9], t1[9], t2[9];
    for (int i = 0; i < 4; ++i) {
        if (dag[i])
            mat3_dag(m[i], f[i]);
        else
            memcpy(f[i], m[i], sizeof(f[i]));
    }
    mat3_mul(f[0], f[1], t1);
    mat3_mul(t1, f[2], t2);
    mat3_mul(t2, f[3], c);
}

static long shift2(const int L[4], long s, int mu, int a, int nu, int b) {
    long t = s;
    if (a) t = neighbour(L, t, mu, a);
    if (b) t = neighbour(L, t, nu, b);
    return t;
}

/*
 * Clover field strength at site s in the (mu, nu) plane:
 *   Q = sum of the four plaquette leaves that start and end at s, each
 *       traversed mu-then-nu (counter-clockwise);
 *   F = (Q - Q^H) / (8i), made traceless.
 */
static void field_strength(const int L[4], const cplx *U, long s, int mu, int nu, cplx F[9]) {
    cplx Q[9] = {0}, leaf[9];
    {
        const cplx *m[4] = {link(U, s, mu), link(U, shift2(L, s, mu, 1, nu, 0), nu),
                            link(U, shift2(L, s, mu, 0, nu, 1), mu), link(U, s, nu)};
        const int d[4] = {0, 0, 1, 1};
        path4(m, d, leaf);
        for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
    }
    {
        const cplx *m[4] = {link(U, s, nu), link(U, shift2(L, s, mu, -1, nu, 1), mu),
                            link(U, shift2(L, s, mu, -1, nu, 0), nu),
                            link(U, shift2(L, s, mu, -1, nu, 0), mu)};
        const int d[4] = {0, 1, 1, 0};
        path4(m, d, leaf);
        for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
    }
    {
        const cplx *m[4] = {link(U, shift2(L, s, mu, -1, nu, 0), mu),
                            link(U, shift2(L, s, mu, -1, nu, -1), nu),
                            link(U, shift2(L, s, mu, -1, nu, -1), mu),
                            link(U, shift2(L, s, mu, 0, nu, -1), nu)};
        const int d[4] = {1, 1, 0, 0};
        path4(m, d, leaf);
        for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
    }
    {
        const cplx *m[4] = {link(U, shift2(L, s, mu, 0, nu, -1), nu),
                            link(U, shift2(L, s, mu, 0, nu, -1), mu),
                            link(U, shift2(L, s, mu, 1, nu, -1), nu), link(U, s, mu)};
        const int d[4] = {1, 0, 0, 1};
        path4(m, d, leaf);
        for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / (8.0 * I);
    const cplx tr = (F[0] + F[4] + F[8]) / 3.0;
    F[0] -= tr;
    F[4] -= tr;
    F[8] -= tr;
}

void oracle_field_strength(const int L[4], const double *U, int mu, int nu, double *F) {
    const long V = volume(L);
    for (long s = 0; s < V; ++s) field_strength(L, (const cplx *)U, s, mu, nu, (cplx *)F + s * 9);
}

/*
 * Clover matrix per site (12x12, row/col index = spin*3 + colour):
 *   A(x) = 1 - kappa c_sw sum_{mu<nu} sigma_mu,nu (x) F_mu,nu(x),
 *   sigma_mu,nu = (i/2) [g_mu, g_nu].
 */
void oracle_clover(const int L[4], double kappa, double csw, const double *Ud, double *Ad) {
    const cplx *U = (const cplx *)Ud;
    cplx *A = (cplx *)Ad;
    const long V = volume(L);
    cplx sigma[4][4][16];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k)
                        c += GAMMA[mu][i][k] * GAMMA[nu][k][j] - GAMMA[nu][i][k] * GAMMA[mu][k][j];
                    sigma[mu][nu][i * 4 + j] = 0.5 * I * c;
                }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        cplx *a = A + s * 144;
        for (int k = 0; k < 144; ++k) a[k] = 0;
        for (int k = 0; k < 12; ++k) a[k * 12 + k] = 1.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx F[9];
                field_strength(L, U, s, mu, nu, F);
                for (int si = 0; si < 4; ++si)
                    for (int sj = 0; sj < 4; ++sj)
                        for (int ci = 0; ci < 3; ++ci)
                            for (int cj = 0; cj < 3; ++cj)
                                a[(si * 3 + ci) * 12 + sj * 3 + cj] -=
                                    kappa * csw * sigma[mu][nu][si * 4 + sj] * F[ci * 3 + cj];
            }
    }
}

/*
 * (M in)(x) at a list of sites only: A(x) in(x) - kappa (D in)(x), with the clover
 * matrix A(x) (csw != 0) assembled at each listed site from its field strengths, as
 * in oracle_clover.  dagger selects M^H = A - kappa D^H.
 */
void oracle_apply_M_sites(const int L[4], double kappa, double csw, const double *bc,
                          const double *Ud, const double *ind, const long *sites, long n,
                          double *outd, int dagger) {
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    cplx sigma[4][4][16];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k)
                        c += GAMMA[mu][i][k] * GAMMA[nu][k][j] - GAMMA[nu][i][k] * GAMMA[mu][k][j];
                    sigma[mu][nu][i * 4 + j] = 0.5 * I * c;
                }
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        const long s = sites[k];
        cplx h[12], a[144];
        hop_site(L, bc, U, in, s, h, dagger);
        for (int q = 0; q < 144; ++q) a[q] = 0;
        for (int q = 0; q < 12; ++q) a[q * 12 + q] = 1.0;
        if (csw != 0.0)
            for (int mu = 0; mu < 4; ++mu)
                for (int nu = mu + 1; nu < 4; ++nu) {
                    cplx F[9];
                    field_strength(L, U, s, mu, nu, F);
                    for (int si = 0; si < 4; ++si)
                        for (int sj = 0; sj < 4; ++sj)
                            for (int ci = 0; ci < 3; ++ci)
                                for (int cj = 0; cj < 3; ++cj)
                                    a[(si * 3 + ci) * 12 + sj * 3 + cj] -=
                                        kappa * csw * sigma[mu][nu][si * 4 + sj] * F[ci * 3 + cj];
                }
        for (int i = 0; i < 12; ++i) {
            cplx v = 0;
            for (int j = 0; j < 12; ++j) v += a[i * 12 + j] * in[s * 12 + j];
            out[k * 12 + i] = v - kappa * h[i];
        }
    }
}

/* per-site inverse of a 12x12 matrix field by Gauss-Jordan with partial pivoting; returns
 * 0, or -1 if a pivot vanished */
int oracle_site_inverse(long nsites, const double *Ad, double *Bd) {
    const cplx *A = (const cplx *)Ad;
    cplx *B = (cplx *)Bd;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long s = 0; s < nsites; ++s) {
        cplx m[12][24];
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 24; ++j)
                m[i][j] = j < 12 ? A[s * 144 + i * 12 + j] : (j - 12 == i ? 1.0 : 0.0);
        for (int c = 0; c < 12; ++c) {
            int p = c;
            for (int r = c + 1; r < 12; ++r)
                if (cabs(m[r][c]) > cabs(m[p][c])) p = r;
            if (cabs(m[p][c]) == 0.0) {
                bad = 1;
                break;
            }
            if (p != c)
                for (int j = 0; j < 24; ++j) {
                    cplx t = m[c][j];
                    m[c][j] = m[p][j];
                    m[p][j] = t;
                }
            const cplx piv = m[c][c];
            for (int j = 0; j < 24; ++j) m[c][j] /= piv;
            for (int r = 0; r < 12; ++r) {
                if (r == c) continue;
                const cplx f = m[r][c];
                for (int j = 0; j < 24; ++j) m[r][j] -= f * m[c][j];
            }
        }
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) B[s * 144 + i * 12 + j] = m[i][12 + j];
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ CG */

static double norm2(const cplx *v, long n) {
    double s = 0;
    for (long k = 0; k < n; ++k) s += creal(v[k]) * creal(v[k]) + cimag(v[k]) * cimag(v[k]);
    return s;
}

static cplx dotc(const cplx *a, const cplx *b, long n) {
    cplx s = 0;
    for (long k = 0; k < n; ++k) s += conj(a[k]) * b[k];
    return s;
}

typedef struct {
    const int *L;
    double kappa;
    const double *bc, *U, *A, *Ainv;
    int system; /* 0: M^H M on the full lattice; 1: S^H S on even sites */
} normal_op;

static void apply_normal(const normal_op *op, const cplx *in, cplx *out, cplx *tmp) {
    if (op->system == 0) {
        oracle_apply_M(op->L, op->kappa, op->bc, op->U, op->A, (const double *)in, (double *)tmp, 0);
        oracle_apply_M(op->L, op->kappa, op->bc, op->U, op->A, (const double *)tmp, (double *)out, 1);
    } else {
        oracle_apply_schur(op->L, op->kappa, op->bc, op->U, op->A, op->Ainv, (const double *)in,
                           (double *)tmp, 0);
        oracle_apply_schur(op->L, op->kappa, op->bc, op->U, op->A, op->Ainv, (const double *)tmp,
                           (double *)out, 1);
    }
}

/*
 * Conjugate gradient (Hestenes-Stiefel) on the Hermitian positive-definite
 * normal operator N = M^H M (system 0) or S^H S (system 1), from x0 = 0:
 *   r = b, p = r, rho = <r,r>
 *   repeat: q = N p; alpha = rho / <p,q>; x += alpha p; r -= alpha q;
 *           rho' = <r,r>; stop if sqrt(rho'/<b,b>) <= tol; p = r + (rho'/rho) p
 * With fixed_iters > 0 exactly that many iterations run and tol is ignored.
 * Returns the iteration count, or -1 when max_iter is reached unconverged.
 * true_res (if non-NULL) receives ||b - N x|| / ||b||, recomputed from x.
 */
int oracle_cg(const int L[4], double kappa, const double *bc, const double *U, const double *A,
              const double *Ainv, int system, const double *bd, double *xd, double tol,
              int max_iter, int fixed_iters, double *true_res) {
    const long n = volume(L) * 12;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    normal_op op = {L, kappa, bc, U, A, Ainv, system};
    memcpy(r, b, sizeof(cplx) * n);
    if (system == 1) mask_parity(L, r, 0);
    for (long k = 0; k < n; ++k) x[k] = 0;
    memcpy(p, r, sizeof(cplx) * n);
    const double bb = norm2(r, n);
    double rho = bb;
    int it = 0, converged = 0;
    const int limit = fixed_iters > 0 ? fixed_iters : max_iter;
    if (bb == 0.0) converged = 1;
    while (!converged && it < limit) {
        apply_normal(&op, p, q, tmp);
        const double pq = creal(dotc(p, q, n));
        const double alpha = rho / pq;
        for (long k = 0; k < n; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
        }
        const double rho1 = norm2(r, n);
        ++it;
        if (fixed_iters <= 0 && sqrt(rho1 / bb) <= tol) converged = 1;
        const double beta = rho1 / rho;
        for (long k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        rho = rho1;
    }
    if (true_res) {
        apply_normal(&op, x, q, tmp);
        memcpy(r, b, sizeof(cplx) * n);
        if (system == 1) mask_parity(L, r, 0);
        for (long k = 0; k < n; ++k) r[k] -= q[k];
        *true_res = bb > 0 ? sqrt(norm2(r, n) / bb) : 0.0;
    }
    free(r);
    free(p);
    free(q);
    free(tmp);
    if (fixed_iters > 0) return it;
    return converged ? it : -1;
}

/* ------------------------------------------------------------------- force */

/*
 * HMC fermion force of S = phi^H (M^H M)^{-1} phi (plain Wilson M) given
 * X = (M^H M)^{-1} phi and Y = M X.  From dS = -2 Re[Y^H dM X] and
 * dM = -kappa dD, the terms of D that contain U_mu(x) give, per link,
 *   G = 2 kappa conj(e+_mu(x)) sum_spin [ ((1-g_mu) Y(x))_s X(x+mu)_s^H
 *                                        + X(x)_s ((1+g_mu) Y(x+mu))_s^H ]
 * which is dS/dRe U + i dS/dIm U (mode 0).  Mode 1 returns the traceless
 * Hermitian F with dS/de = Tr(H F) for U -> exp(i e H) U:
 *   W = U G^H, F = i (W - W^H) / 2 minus its trace / 3.
 */
void oracle_force(const int L[4], double kappa, const double *bc, const double *Ud,
                  const double *Xd, const double *Yd, double *Fd, int mode) {
    const cplx *U = (const cplx *)Ud, *X = (const cplx *)Xd, *Y = (const cplx *)Yd;
    cplx *F = (cplx *)Fd;
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int x[4];
        site_coords(L, s, x);
        for (int mu = 0; mu < 4; ++mu) {
            const long sf = neighbour(L, s, mu, +1);
            const cplx phase = bc[2 * mu] + I * bc[2 * mu + 1];
            const cplx ef = (x[mu] == L[mu] - 1) ? phase : 1.0;
            cplx a[12], b[12];
            for (int sp = 0; sp < 4; ++sp)
                for (int c = 0; c < 3; ++c) {
                    cplx ga = 0, gb = 0;
                    for (int t = 0; t < 4; ++t) {
                        ga += GAMMA[mu][sp][t] * Y[s * 12 + t * 3 + c];
                        gb += GAMMA[mu][sp][t] * Y[sf * 12 + t * 3 + c];
                    }
                    a[sp * 3 + c] = Y[s * 12 + sp * 3 + c] - ga;
                    b[sp * 3 + c] = Y[sf * 12 + sp * 3 + c] + gb;
                }
            cplx G[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    cplx v = 0;
                    for (int sp = 0; sp < 4; ++sp)
                        v += a[sp * 3 + i] * conj(X[sf * 12 + sp * 3 + j]) +
                             X[s * 12 + sp * 3 + i] * conj(b[sp * 3 + j]);
                    G[i * 3 + j] = 2.0 * kappa * conj(ef) * v;
                }
            cplx *out = F + (s * 4 + mu) * 9;
            if (mode == 0) {
                memcpy(out, G, sizeof(G));
            } else {
                cplx Gh[9], W[9];
                mat3_dag(G, Gh);
                mat3_mul(link(U, s, mu), Gh, W);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        out[i * 3 + j] = 0.5 * I * (W[i * 3 + j] - conj(W[j * 3 + i]));
                const cplx tr = (out[0] + out[4] + out[8]) / 3.0;
                out[0] -= tr;
                out[4] -= tr;
                out[8] -= tr;
            }
        }
    }
}

/* ------------------------------------------------------------------ helpers */

/* average over plaquettes of Re Tr P / 3 */
double oracle_plaquette(const int L[4], const double *Ud) {
    const cplx *U = (const cplx *)Ud;
    const long V = volume(L);
    double sum = 0;
    for (long s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                const cplx *m[4] = {link(U, s, mu), link(U, neighbour(L, s, mu, 1), nu),
                                    link(U, neighbour(L, s, nu, 1), mu), link(U, s, nu)};
                const int d[4] = {0, 0, 1, 1};
                cplx P[9];
                path4(m, d, P);
                sum += creal(P[0] + P[4] + P[8]) / 3.0;
            }
    return sum / (6.0 * V);
}

void oracle_gamma(int mu, double *out) {
    for (int i = 0; i < 16; ++i) {
        out[2 * i] = creal(GAMMA[mu][i / 4][i % 4]);
        out[2 * i + 1] = cimag(GAMMA[mu][i / 4][i % 4]);
    }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
