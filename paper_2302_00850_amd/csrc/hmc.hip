// Kernels of the HMC molecular-dynamics step (hybrid Monte Carlo: the gauge-field
// generation algorithm the paper lists, after Duane et al.) on canonical FP64 fields
// U[site][mu][3][3] and traceless Hermitian momenta P of the same layout:
//
//   gauge force   F_mu(x) = -(beta/3) P_TH[i (W - W^H) / 2],  W = U_mu(x) A_mu(x), A the
//                 sum of the six staples, so that dS_g/de = Tr(H F) along
//                 U -> exp(i e H) U for S_g = beta sum_plaq (1 - Re Tr U_plaq / 3)
//   momentum      P -= eps (F1 + F2)
//   link update   U <- exp(i eps P) U (scaling and squaring of a Taylor series)
//   reductions    sum of Re Tr U_plaq, sum of Tr P^2, Re <a, b>: per-block partials
//                 in a fixed-shape LDS tree, then the block-order reduce launch.
//
// One lane per link (or per site for the plaquette sum), grid-stride loops.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

using C = cpx<double>;

// grid cap of the grid-stride kernels (also the partial count of their reductions)
constexpr int kHmcGrid = 4096;
static_assert(kHmcGrid <= kRedMaxBlocks, "reduction partials");

struct M3 {
    C a[3][3];
};

__device__ __forceinline__ C conj(C a) { return {a.x, -a.y}; }

__device__ __forceinline__ M3 ld3(const C *p) {
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.a[i][j] = p[3 * i + j];
    return m;
}

__device__ __forceinline__ void st3(C *p, const M3 &m) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) p[3 * i + j] = m.a[i][j];
}

// A B, A B^H, A^H B
__device__ __forceinline__ M3 mm(const M3 &A, const M3 &B) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmul(A.a[i][0], B.a[0][j]);
            s = cmadd(s, A.a[i][1], B.a[1][j]);
            r.a[i][j] = cmadd(s, A.a[i][2], B.a[2][j]);
        }
    return r;
}
__device__ __forceinline__ M3 mmd(const M3 &A, const M3 &B) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmul(A.a[i][0], conj(B.a[j][0]));
            s = cmadd(s, A.a[i][1], conj(B.a[j][1]));
            r.a[i][j] = cmadd(s, A.a[i][2], conj(B.a[j][2]));
        }
    return r;
}
__device__ __forceinline__ M3 mdm(const M3 &A, const M3 &B) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmul(conj(A.a[0][i]), B.a[0][j]);
            s = cmadd(s, conj(A.a[1][i]), B.a[1][j]);
            r.a[i][j] = cmadd(s, conj(A.a[2][i]), B.a[2][j]);
        }
    return r;
}

__device__ __forceinline__ void coords(const Geom &g, uint32_t s, int x[4]) {
    uint32_t q = s;
    x[0] = (int)(q % (uint32_t)g.L[0]);
    q /= (uint32_t)g.L[0];
    x[1] = (int)(q % (uint32_t)g.L[1]);
    q /= (uint32_t)g.L[1];
    x[2] = (int)(q % (uint32_t)g.L[2]);
    x[3] = (int)(q / (uint32_t)g.L[2]);
}

// lexicographic site of x + d mu (d = +-1), periodic
__device__ __forceinline__ uint32_t step(const Geom &g, const int x[4], int mu, int d,
                                         int y[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] += d;
    if (y[mu] == g.L[mu]) y[mu] = 0;
    if (y[mu] < 0) y[mu] = g.L[mu] - 1;
    return (uint32_t)(y[0] + g.L[0] * (y[1] + g.L[1] * (y[2] + g.L[2] * y[3])));
}

__device__ __forceinline__ const C *link(const C *U, uint32_t s, int mu) {
    return U + ((size_t)s * 4 + (size_t)mu) * 9;
}

// Gauge force F_mu(x) = -(beta/3) traceless part of i (W - W^H) / 2 with W = U_mu(x) A and A
// the sum of the six staples around U_mu(x).  Three lanes per link, one per direction
// nu != mu, each forming its upper and lower staple (six link loads, about a third of
// the registers of one lane doing all six staples, so three times the waves hide the
// scattered link loads); the three partial sums meet in LDS and the link's first lane
// adds them in nu order and finishes W and F.  A block covers 64 links per pass.
constexpr int kGfLinks = 64;

__global__ void __launch_bounds__(3 * kGfLinks) gauge_force_kernel(const Geom g,
                                                                   const C *__restrict__ U,
                                                                   C *__restrict__ F,
                                                                   double beta) {
    __shared__ M3 part[3 * kGfLinks];
    const uint32_t nlinks = 8u * (uint32_t)g.Vh;
    const int k = threadIdx.x % 3;
    const int lk = threadIdx.x / 3;
    // the pass count is the same for every lane of the block (barriers inside)
    for (uint32_t base = blockIdx.x * kGfLinks; base < nlinks; base += gridDim.x * kGfLinks) {
        const uint32_t l = base + (uint32_t)lk;
        const bool valid = l < nlinks;
        const uint32_t s = l >> 2;
        const int mu = (int)(l & 3u);
        int x[4], y[4], z[4], w[4];
        if (valid) {
            coords(g, s, x);
            const uint32_t sp = step(g, x, mu, 1, y);  // x + mu
            const int nu = k + (k >= mu ? 1 : 0);
            const uint32_t sn = step(g, x, nu, 1, w);    // x + nu
            const uint32_t sm = step(g, x, nu, -1, w);   // x - nu
            const uint32_t spm = step(g, y, nu, -1, z);  // x + mu - nu
            // upper: U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H, parked in LDS before the lower
            // staple's loads are issued (the empty asm keeps them apart), so that one
            // staple's matrices are live at a time
            part[threadIdx.x] =
                mmd(mmd(ld3(link(U, sp, nu)), ld3(link(U, sn, mu))), ld3(link(U, s, nu)));
            asm volatile("" ::: "memory");
            // lower: U_nu(x+mu-nu)^H U_mu(x-nu)^H U_nu(x-nu)
            //     = (U_mu(x-nu) U_nu(x+mu-nu))^H U_nu(x-nu)
            const M3 low = mdm(mm(ld3(link(U, sm, mu)), ld3(link(U, spm, nu))),
                               ld3(link(U, sm, nu)));
            M3 &st = part[threadIdx.x];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    st.a[i][j] = {st.a[i][j].x + low.a[i][j].x, st.a[i][j].y + low.a[i][j].y};
        }
        __syncthreads();
        if (valid && k == 0) {
            M3 A;
            const M3 &p0 = part[threadIdx.x], &p1 = part[threadIdx.x + 1], &p2 = part[threadIdx.x + 2];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    A.a[i][j] = {(p0.a[i][j].x + p1.a[i][j].x) + p2.a[i][j].x,
                                 (p0.a[i][j].y + p1.a[i][j].y) + p2.a[i][j].y};
            const M3 W = mm(ld3(link(U, s, mu)), A);
            // X = i (W - W^H) / 2, traceless, times -(beta / 3)
            M3 X;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const C d = {W.a[i][j].x - W.a[j][i].x, W.a[i][j].y + W.a[j][i].y};
                    X.a[i][j] = {-0.5 * d.y, 0.5 * d.x};  // i d / 2
                }
            const double tr = (X.a[0][0].x + X.a[1][1].x + X.a[2][2].x) / 3.0;
            const double f = -beta / 3.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                X.a[i][i].x -= tr;
                X.a[i][i].y = 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j) X.a[i][j] = {f * X.a[i][j].x, f * X.a[i][j].y};
            }
            st3(F + (size_t)l * 9, X);
        }
        __syncthreads();  // part is reused by the next pass
    }
}

__global__ void __launch_bounds__(256) momentum_kernel(C *__restrict__ P,
                                                       const C *__restrict__ F1,
                                                       const C *__restrict__ F2, double eps,
                                                       size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
        C f = F1[k];
        if (F2) f = {f.x + F2[k].x, f.y + F2[k].y};
        P[k] = {fma(-eps, f.x, P[k].x), fma(-eps, f.y, P[k].y)};
    }
}

// exp(X) for X = i eps P: halve until the 1-norm is at most 1/2, Taylor series to 16th
// order (truncation below 1e-19 there), square back.
__device__ __forceinline__ M3 expi3(const M3 &P, double eps) {
    M3 X;
    double nrm = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double c = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            X.a[i][j] = {-eps * P.a[i][j].y, eps * P.a[i][j].x};
            c += sqrt(X.a[i][j].x * X.a[i][j].x + X.a[i][j].y * X.a[i][j].y);
        }
        nrm = fmax(nrm, c);
    }
    int sq = 0;
    double scale = 1.0;
    while (nrm * scale > 0.5 && sq < 60) {
        scale *= 0.5;
        ++sq;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) X.a[i][j] = {scale * X.a[i][j].x, scale * X.a[i][j].y};
    // Horner: E = I + X/1 (I + X/2 (I + ... (I + X/16)))
    M3 E;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) E.a[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    for (int k = 16; k >= 1; --k) {
        M3 T = mm(X, E);
        const double r = 1.0 / k;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                E.a[i][j] = {(i == j ? 1.0 : 0.0) + r * T.a[i][j].x, r * T.a[i][j].y};
    }
    for (int k = 0; k < sq; ++k) E = mm(E, E);
    return E;
}

// Rows re-orthonormalised (Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)): the
// SU(3) matrix nearest to a link that rounding has moved off the group by O(1e-16).
__device__ __forceinline__ M3 reunitarise(M3 m) {
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += norm2(m.a[0][j]);
    const double i0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.a[0][j] = {i0 * m.a[0][j].x, i0 * m.a[0][j].y};
    C d = {0.0, 0.0};  // <row0, row1>
#pragma unroll
    for (int j = 0; j < 3; ++j) d = cmadd(d, conj(m.a[0][j]), m.a[1][j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.a[1][j] = m.a[1][j] - cmul(d, m.a[0][j]);
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n1 += norm2(m.a[1][j]);
    const double i1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.a[1][j] = {i1 * m.a[1][j].x, i1 * m.a[1][j].y};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const C c = cmul(m.a[0][k1], m.a[1][k2]) - cmul(m.a[0][k2], m.a[1][k1]);
        m.a[2][k] = conj(c);
    }
    return m;
}

// U <- exp(i eps P) U, re-unitarised: without the projection, rounding moves the links
// off SU(3) by about 1e-16 per update, which over many trajectories would exceed the
// SU(3) check that the compressed (12-real) link formats require.
__global__ void __launch_bounds__(256) link_update_kernel(C *__restrict__ U,
                                                          const C *__restrict__ P, double eps,
                                                          size_t nlinks) {
    for (size_t l = (size_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlinks;
         l += (size_t)gridDim.x * blockDim.x) {
        const M3 E = expi3(ld3(P + l * 9), eps);
        st3(U + l * 9, reunitarise(mm(E, ld3(U + l * 9))));
    }
}

// ---------------------------------------------------------------- APE smearing
// (the smeared links of the fat-link irrelevant clover operator)

__device__ __forceinline__ C cdiv(C a, C b) {
    const double d = 1.0 / (b.x * b.x + b.y * b.y);
    return {(a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d};
}

__device__ __forceinline__ C det3(const M3 &m) {
    const C c0 = cmul(m.a[1][1], m.a[2][2]) - cmul(m.a[1][2], m.a[2][1]);
    const C c1 = cmul(m.a[1][2], m.a[2][0]) - cmul(m.a[1][0], m.a[2][2]);
    const C c2 = cmul(m.a[1][0], m.a[2][1]) - cmul(m.a[1][1], m.a[2][0]);
    return cmadd(cmadd(cmul(m.a[0][0], c0), m.a[0][1], c1), m.a[0][2], c2);
}

// X^{-H} = adj(X)^H / conj(det X), adj the adjugate (transposed cofactors)
__device__ __forceinline__ M3 inv_dag(const M3 &X, C det) {
    M3 cof;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof.a[i][j] = cmul(X.a[i1][j1], X.a[i2][j2]) - cmul(X.a[i1][j2], X.a[i2][j1]);
        }
    // (adj X)^H = conj(cof); divided by conj(det)
    M3 r;
    const C cd = conj(det);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.a[i][j] = cdiv(conj(cof.a[i][j]), cd);
    return r;
}

// The SU(3) matrix nearest to V: the unitary polar factor W (V = W H, H Hermitian
// positive) by Newton's iteration X <- (g X + X^{-H} / g) / 2 with the determinant scaling
// g = |det X|^{-1/3} (quadratic convergence; stopped when an iteration changes no entry
// by more than 1e-15), then det(W)^{-1/3} with the principal cube root.
__device__ M3 project_su3(const M3 &V) {
    M3 X = V;
    for (int it = 0; it < 40; ++it) {
        const C det = det3(X);
        const double g = pow(sqrt(det.x * det.x + det.y * det.y), -1.0 / 3.0);
        const M3 Y = inv_dag(X, det);
        double change = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const C n = {0.5 * (g * X.a[i][j].x + Y.a[i][j].x / g),
                             0.5 * (g * X.a[i][j].y + Y.a[i][j].y / g)};
                change = fmax(change, fmax(fabs(n.x - X.a[i][j].x), fabs(n.y - X.a[i][j].y)));
                X.a[i][j] = n;
            }
        if (change <= 1e-15) break;
    }
    const C d = det3(X);
    const double th = atan2(d.y, d.x) / 3.0;
    const C ph = {cos(th), -sin(th)};  // det^{-1/3}
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) X.a[i][j] = cmul(X.a[i][j], ph);
    return X;
}

// One APE sweep: V_mu(x) = (1 - alpha) U_mu(x) + (alpha / 6) sum over nu != mu of the
// staples U_nu(x) U_mu(x+nu) U_nu(x+mu)^H and U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu), then
// projected to SU(3).  Periodic links; reads U, writes Out (no aliasing).
__global__ void __launch_bounds__(256) ape_kernel(const Geom g, const C *__restrict__ U,
                                                  C *__restrict__ Out, double alpha) {
    const uint32_t V = 2u * (uint32_t)g.Vh;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < 4u * V;
         t += gridDim.x * blockDim.x) {
        const uint32_t s = t >> 2;
        const int mu = (int)(t & 3u);
        int x[4], y[4], w[4], z[4];
        coords(g, s, x);
        const uint32_t sp = step(g, x, mu, 1, y);  // x + mu
        M3 S;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) S.a[i][j] = C{0.0, 0.0};
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            const uint32_t sn = step(g, x, nu, 1, w);    // x + nu
            const uint32_t sm = step(g, x, nu, -1, w);   // x - nu
            const uint32_t smp = step(g, w, mu, 1, z);   // x - nu + mu
            const M3 up = mmd(mm(ld3(link(U, s, nu)), ld3(link(U, sn, mu))), ld3(link(U, sp, nu)));
            const M3 lo = mm(mdm(ld3(link(U, sm, nu)), ld3(link(U, sm, mu))), ld3(link(U, smp, nu)));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) S.a[i][j] = S.a[i][j] + up.a[i][j] + lo.a[i][j];
        }
        const M3 Um = ld3(link(U, s, mu));
        M3 Vm;
        const double a0 = 1.0 - alpha, a1 = alpha / 6.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Vm.a[i][j] = {fma(a1, S.a[i][j].x, a0 * Um.a[i][j].x),
                              fma(a1, S.a[i][j].y, a0 * Um.a[i][j].y)};
        st3(Out + (size_t)t * 9, project_su3(Vm));
    }
}

// fixed-shape LDS tree over the 256 lanes of a block; lane 0 writes the partial
__device__ __forceinline__ void block_partial(double v, double *partial) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) plaquette_kernel(const Geom g, const C *__restrict__ U,
                                                        double *__restrict__ partial) {
    const uint32_t V = 2u * (uint32_t)g.Vh;
    double acc = 0.0;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < V;
         s += gridDim.x * blockDim.x) {
        int x[4], y[4], z[4];
        coords(g, s, x);
        for (int mu = 0; mu < 4; ++mu) {
            const uint32_t sp = step(g, x, mu, 1, y);
            for (int nu = mu + 1; nu < 4; ++nu) {
                const uint32_t sn = step(g, x, nu, 1, z);
                // Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H
                const M3 a = mm(ld3(link(U, s, mu)), ld3(link(U, sp, nu)));
                const M3 c = mmd(a, ld3(link(U, sn, mu)));
                const M3 d = mmd(c, ld3(link(U, s, nu)));
                acc += d.a[0][0].x + d.a[1][1].x + d.a[2][2].x;
            }
        }
    }
    block_partial(acc, partial);
}

__global__ void __launch_bounds__(256) sqnorm_kernel(const C *__restrict__ a, size_t n,
                                                     double *__restrict__ partial) {
    double acc = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        acc = fma(a[k].x, a[k].x, fma(a[k].y, a[k].y, acc));
    block_partial(acc, partial);
}

__global__ void __launch_bounds__(256) redot_kernel(const C *__restrict__ a,
                                                    const C *__restrict__ b, size_t n,
                                                    double *__restrict__ partial) {
    double acc = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        acc = fma(a[k].x, b[k].x, fma(a[k].y, b[k].y, acc));
    block_partial(acc, partial);
}

int grid_for(size_t n) {
    const size_t g = (n + 255) / 256;
    return (int)std::max<size_t>(1, std::min<size_t>(g, kHmcGrid));
}

}  // namespace

hipError_t launch_gauge_force(const Geom &g, const void *U, void *F, double beta,
                              hipStream_t st) {
    const size_t n = (size_t)8 * g.Vh;
    const size_t blocks = (n + kGfLinks - 1) / kGfLinks;
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(blocks, 65536));
    hipLaunchKernelGGL(gauge_force_kernel, dim3(grid), dim3(3 * kGfLinks), 0, st, g,
                       (const C *)U, (C *)F, beta);
    return hipGetLastError();
}

hipError_t launch_momentum_update(void *P, const void *F1, const void *F2, double eps,
                                  size_t nlinks, hipStream_t st) {
    const size_t n = nlinks * 9;
    hipLaunchKernelGGL(momentum_kernel, dim3(grid_for(n)), dim3(256), 0, st, (C *)P,
                       (const C *)F1, (const C *)F2, eps, n);
    return hipGetLastError();
}

hipError_t launch_link_update(void *U, const void *P, double eps, size_t nlinks,
                              hipStream_t st) {
    hipLaunchKernelGGL(link_update_kernel, dim3(grid_for(nlinks)), dim3(256), 0, st, (C *)U,
                       (const C *)P, eps, nlinks);
    return hipGetLastError();
}

hipError_t launch_ape_sweep(const Geom &g, const void *U, void *Out, double alpha,
                            hipStream_t st) {
    const size_t n = (size_t)8 * g.Vh;
    hipLaunchKernelGGL(ape_kernel, dim3(grid_for(n)), dim3(256), 0, st, g, (const C *)U, (C *)Out,
                       alpha);
    return hipGetLastError();
}

hipError_t launch_plaquette_sum(const Geom &g, const void *U, double *partial, double *result,
                                hipStream_t st) {
    const int grid = grid_for((size_t)2 * g.Vh);
    hipLaunchKernelGGL(plaquette_kernel, dim3(grid), dim3(256), 0, st, g, (const C *)U,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 1, result, st);
}

hipError_t launch_sqnorm(const void *a, size_t n, double *partial, double *result,
                         hipStream_t st) {
    const int grid = grid_for(n);
    hipLaunchKernelGGL(sqnorm_kernel, dim3(grid), dim3(256), 0, st, (const C *)a, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 1, result, st);
}

hipError_t launch_redot(const void *a, const void *b, size_t n, double *partial, double *result,
                        hipStream_t st) {
    const int grid = grid_for(n);
    hipLaunchKernelGGL(redot_kernel, dim3(grid), dim3(256), 0, st, (const C *)a, (const C *)b, n,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 1, result, st);
}

}  // namespace cola
