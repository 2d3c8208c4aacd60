// Clover term: field strength from the four plaquette leaves around each site,
// assembled into the two Hermitian 6x6 chiral blocks of
//   A = 1 - kappa c_sw sum_{mu<nu} sigma_mu,nu F_mu,nu,
// and the per-block inverse by Cholesky factorisation (FP64).
//
// In the chiral basis sigma_mu,nu = (i/2)[g_mu, g_nu] is block diagonal; with
// Pauli matrices s1, s2, s3 acting on the two spins of a block,
//   upper block (spins 0,1): s3 (F_xy - F_zt) + s2 (F_xz + F_yt) + s1 (F_yz - F_xt)
//   lower block (spins 2,3): s3 (F_xy + F_zt) + s2 (F_xz - F_yt) + s1 (F_yz + F_xt)
// so each block is [[1 - k B3, -k (B1 - i B2)], [-k (B1 + i B2), 1 + k B3]] with
// k = kappa c_sw and B1..B3 the 3x3 colour combinations above.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

using C = cpx<double>;

struct M3 {
    C m[9];
};

__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmul(a.m[i * 3], b.m[j]);
            s = cmadd(s, a.m[i * 3 + 1], b.m[3 + j]);
            s = cmadd(s, a.m[i * 3 + 2], b.m[6 + j]);
            c.m[i * 3 + j] = s;
        }
    return c;
}

__device__ __forceinline__ M3 dag(const M3 &a) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.m[i * 3 + j] = {a.m[j * 3 + i].x, -a.m[j * 3 + i].y};
    return c;
}

struct Lat {
    int L[4];
    const C *U;
    __device__ uint32_t idx(const int x[4]) const {
        return (uint32_t)(x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3])));
    }
    // link U_mu at x + a*e_mu' + b*e_nu' (periodic)
    __device__ M3 link(const int x[4], int mu, int d1, int s1, int d2, int s2) const {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[d1] = (y[d1] + s1 + L[d1]) % L[d1];
        y[d2] = (y[d2] + s2 + L[d2]) % L[d2];
        M3 r;
        const C *p = U + ((size_t)idx(y) * 4 + mu) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) r.m[k] = p[k];
        return r;
    }
};

// F_mu,nu(x) = traceless part of (Q - Q^H) / (8i), Q = sum of the four leaves
__device__ M3 field_strength(const Lat &lat, const int x[4], int mu, int nu) {
    M3 q;
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = {0.0, 0.0};
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H
    {
        M3 l = mul(mul(lat.link(x, mu, mu, 0, nu, 0), lat.link(x, nu, mu, 1, nu, 0)),
                   mul(dag(lat.link(x, mu, mu, 0, nu, 1)), dag(lat.link(x, nu, mu, 0, nu, 0))));
        for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
    }
    // leaf 2: U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu)
    {
        M3 l = mul(mul(lat.link(x, nu, mu, 0, nu, 0), dag(lat.link(x, mu, mu, -1, nu, 1))),
                   mul(dag(lat.link(x, nu, mu, -1, nu, 0)), lat.link(x, mu, mu, -1, nu, 0)));
        for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
    }
    // leaf 3: U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu)
    {
        M3 l = mul(mul(dag(lat.link(x, mu, mu, -1, nu, 0)), dag(lat.link(x, nu, mu, -1, nu, -1))),
                   mul(lat.link(x, mu, mu, -1, nu, -1), lat.link(x, nu, mu, 0, nu, -1)));
        for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
    }
    // leaf 4: U_nu(x-nu)^H U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^H
    {
        M3 l = mul(mul(dag(lat.link(x, nu, mu, 0, nu, -1)), lat.link(x, mu, mu, 0, nu, -1)),
                   mul(lat.link(x, nu, mu, 1, nu, -1), dag(lat.link(x, mu, mu, 0, nu, 0))));
        for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + l.m[k];
    }
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // (q_ij - conj(q_ji)) / (8i) = -i/8 (q_ij - conj(q_ji))
            const C d = {q.m[i * 3 + j].x - q.m[j * 3 + i].x, q.m[i * 3 + j].y + q.m[j * 3 + i].y};
            f.m[i * 3 + j] = {d.y / 8.0, -d.x / 8.0};
        }
    const double tr = (f.m[0].x + f.m[4].x + f.m[8].x) / 3.0;  // F Hermitian: real trace
    f.m[0].x -= tr;
    f.m[4].x -= tr;
    f.m[8].x -= tr;
    return f;
}

// Cholesky inverse of a Hermitian positive-definite 6x6 matrix (full storage).
// Returns false if a pivot is not positive.
__device__ bool hpd_inverse6(const C a[36], C inv[36]) {
    C l[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) l[k] = {0.0, 0.0};
    for (int j = 0; j < 6; ++j) {
        double d = a[j * 6 + j].x;
        for (int k = 0; k < j; ++k) d -= norm2(l[j * 6 + k]);
        if (!(d > 0.0)) return false;
        const double ljj = sqrt(d);
        l[j * 6 + j] = {ljj, 0.0};
        for (int i = j + 1; i < 6; ++i) {
            C s = a[i * 6 + j];
            for (int k = 0; k < j; ++k) {
                // s -= l_ik conj(l_jk)
                const C lik = l[i * 6 + k], ljk = l[j * 6 + k];
                s.x -= lik.x * ljk.x + lik.y * ljk.y;
                s.y -= lik.y * ljk.x - lik.x * ljk.y;
            }
            l[i * 6 + j] = {s.x / ljj, s.y / ljj};
        }
    }
    // inverse: solve L L^H X = e_c column by column
    for (int c = 0; c < 6; ++c) {
        C y[6];
        for (int i = 0; i < 6; ++i) {
            C s = {i == c ? 1.0 : 0.0, 0.0};
            for (int k = 0; k < i; ++k) s = s - cmul(l[i * 6 + k], y[k]);
            y[i] = {s.x / l[i * 6 + i].x, s.y / l[i * 6 + i].x};
        }
        for (int i = 5; i >= 0; --i) {
            C s = y[i];
            for (int k = i + 1; k < 6; ++k) s = s - cmul(C{l[k * 6 + i].x, -l[k * 6 + i].y}, inv[k * 6 + c]);
            inv[i * 6 + c] = {s.x / l[i * 6 + i].x, s.y / l[i * 6 + i].x};
        }
    }
    return true;
}

template <typename T>
__device__ void store_block(void *buf, int S, int p, uint32_t i, int blk, const C a[36]) {
    struct alignas(2 * sizeof(T)) pr { T a, b; };
    pr *q = (pr *)buf + ((size_t)(p * 36 + blk * 18)) * S + i;
#pragma unroll
    for (int k = 0; k < 3; ++k) q[(size_t)k * S] = pr{(T)a[(2 * k) * 7].x, (T)a[(2 * k + 1) * 7].x};
    for (int r = 1; r < 6; ++r)
        for (int c = 0; c < r; ++c)
            q[(size_t)(3 + r * (r - 1) / 2 + c) * S] = pr{(T)a[r * 6 + c].x, (T)a[r * 6 + c].y};
}

__global__ void __launch_bounds__(128) clover_build_kernel(const Geom g, const C *__restrict__ U, double kappa, double csw,
                                    void *a64, void *ainv64, void *a32, void *ainv32, int *bad) {
    const uint32_t V = 2u * (uint32_t)g.Vh;
    Lat lat;
    for (int k = 0; k < 4; ++k) lat.L[k] = g.L[k];
    lat.U = U;
    const double kc = kappa * csw;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < V; s += gridDim.x * blockDim.x) {
        int x[4];
        uint32_t t = s;
        x[0] = (int)(t % (uint32_t)g.L[0]);
        t /= (uint32_t)g.L[0];
        x[1] = (int)(t % (uint32_t)g.L[1]);
        t /= (uint32_t)g.L[1];
        x[2] = (int)(t % (uint32_t)g.L[2]);
        x[3] = (int)(t / (uint32_t)g.L[2]);
        const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
        const uint32_t i = s >> 1;
        const M3 fxy = field_strength(lat, x, 0, 1), fxz = field_strength(lat, x, 0, 2);
        const M3 fxt = field_strength(lat, x, 0, 3), fyz = field_strength(lat, x, 1, 2);
        const M3 fyt = field_strength(lat, x, 1, 3), fzt = field_strength(lat, x, 2, 3);
        for (int blk = 0; blk < 2; ++blk) {
            const double sgn = blk == 0 ? -1.0 : 1.0;  // upper: F_xy - F_zt, ...
            C a[36];
            for (int ci = 0; ci < 3; ++ci)
                for (int cj = 0; cj < 3; ++cj) {
                    const int k = ci * 3 + cj;
                    const C b3 = fxy.m[k] + scale(sgn, fzt.m[k]);
                    const C b2 = fxz.m[k] + scale(-sgn, fyt.m[k]);
                    const C b1 = fyz.m[k] + scale(sgn, fxt.m[k]);
                    const double dlt = ci == cj ? 1.0 : 0.0;
                    // [[1 - k B3, -k (B1 - i B2)], [-k (B1 + i B2), 1 + k B3]]
                    a[ci * 6 + cj] = {dlt - kc * b3.x, -kc * b3.y};
                    a[(3 + ci) * 6 + 3 + cj] = {dlt + kc * b3.x, kc * b3.y};
                    const C b1mib2 = {b1.x + b2.y, b1.y - b2.x};
                    const C b1pib2 = {b1.x - b2.y, b1.y + b2.x};
                    a[ci * 6 + 3 + cj] = scale(-kc, b1mib2);
                    a[(3 + ci) * 6 + cj] = scale(-kc, b1pib2);
                }
            C inv[36];
            if (!hpd_inverse6(a, inv)) {
                atomicAdd(bad, 1);
                for (int k = 0; k < 36; ++k) inv[k] = {0.0, 0.0};
            }
            if (a64) store_block<double>(a64, g.S, p, i, blk, a);
            if (ainv64) store_block<double>(ainv64, g.S, p, i, blk, inv);
            if (a32) store_block<float>(a32, g.S, p, i, blk, a);
            if (ainv32) store_block<float>(ainv32, g.S, p, i, blk, inv);
        }
    }
}

}  // namespace

hipError_t launch_clover_build(const Geom &g, const void *U, double kappa, double csw,
                               void *a64, void *ainv64, void *a32, void *ainv32, int *bad,
                               hipStream_t st) {
    const size_t V = (size_t)g.Vh * 2;
    size_t grid = (V + 127) / 128;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(clover_build_kernel, dim3((unsigned)grid), dim3(128), 0, st, g,
                       (const C *)U, kappa, csw, a64, ainv64, a32, ainv32, bad);
    return hipGetLastError();
}

}  // namespace cola
