// HMC fermion force for S = phi^H (M^H M)^{-1} phi with plain Wilson M.
//
// With X = (M^H M)^{-1} phi and Y = M X, varying S gives dS = -2 Re[Y^H dM X]
// and dM = -kappa dD.  The two hopping terms that contain U_mu(x) are the
// forward hop out of x and the backward hop out of x + mu, so one lane per
// link forms
//   G = 2 kappa conj(e+_mu(x)) sum_spin [ ((1 - g_mu) Y(x))_s X(x+mu)_s^H
//                                        + X(x)_s ((1 + g_mu) Y(x+mu))_s^H ]
// (= dS/dRe U + i dS/dIm U).  The Lie-algebra form, for U -> exp(i e H) U,
// is F = traceless part of i (W - W^H) / 2 with W = U G^H.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

using C = cpx<double>;

__global__ void __launch_bounds__(256) force_kernel(const Geom g, const void *gauge, const C *__restrict__ X,
                             const C *__restrict__ Y, C *__restrict__ F, double kappa,
                             Cplx64 ph0, Cplx64 ph1, Cplx64 ph2, Cplx64 ph3, int mode) {
    const uint32_t V = 2u * (uint32_t)g.Vh;
    const Cplx64 phs[4] = {ph0, ph1, ph2, ph3};
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < V * 4u;
         t += gridDim.x * blockDim.x) {
        const uint32_t s = t >> 2;
        const int mu = (int)(t & 3u);
        int x[4];
        uint32_t q = s;
        x[0] = (int)(q % (uint32_t)g.L[0]);
        q /= (uint32_t)g.L[0];
        x[1] = (int)(q % (uint32_t)g.L[1]);
        q /= (uint32_t)g.L[1];
        x[2] = (int)(q % (uint32_t)g.L[2]);
        x[3] = (int)(q / (uint32_t)g.L[2]);
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[mu] = y[mu] + 1 == g.L[mu] ? 0 : y[mu] + 1;
        const uint32_t sf = (uint32_t)(y[0] + g.L[0] * (y[1] + g.L[1] * (y[2] + g.L[2] * y[3])));
        // (1 -+ g_mu) = E E^H with E^H the spin projection (E^H E = 2), so each spin sum
        // runs over the two projected components:
        //   sum_s ((1 - g_mu) Y(x))_s,a conj(X(x+mu)_s,b) = sum_k hY_k,a conj(hXf_k,b),
        //   hY = project_-(Y(x)), hXf = project_-(X(x+mu)); likewise with project_+ for
        //   X(x) and (1 + g_mu) Y(x+mu).  One spinor is loaded at a time.
        const bool bnd = x[mu] == g.L[mu] - 1;
        // 2 kappa conj(e+)
        const C f = bnd ? C{2.0 * kappa * phs[mu].x, -2.0 * kappa * phs[mu].y}
                        : C{2.0 * kappa, 0.0};
        C G[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = C{0.0, 0.0};
        auto load = [](const C *v, uint32_t site, C out[12]) {
#pragma unroll
            for (int c = 0; c < 12; ++c) out[c] = v[(size_t)site * 12 + c];
        };
        auto accumulate = [&](const C ha[6], const C hb[6]) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        G[a * 3 + b] = cjmadd(G[a * 3 + b], hb[k * 3 + b], ha[k * 3 + a]);
        };
        C sp[12], ha[6], hb[6];
        load(Y, s, sp);
        project(mu, -1.0, sp, ha);
        load(X, sf, sp);
        project(mu, -1.0, sp, hb);
        accumulate(ha, hb);
        load(X, s, sp);
        project(mu, 1.0, sp, ha);
        load(Y, sf, sp);
        project(mu, 1.0, sp, hb);
        accumulate(ha, hb);
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = cmul(f, G[k]);
        C *out = F + (size_t)t * 9;
        if (mode == 0) {
#pragma unroll
            for (int k = 0; k < 9; ++k) out[k] = G[k];
            continue;
        }
        const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
        C u[3][3];
        load_link<LinkFmt::F64_18, double, false>(gauge, g.S, p, mu, s >> 1, u);
        // W = U G^H
        C W[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                C acc = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) acc = cjmadd(acc, G[b * 3 + k], u[a][k]);
                W[a * 3 + b] = acc;
            }
        // i (W - W^H) / 2
        C Fm[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const C d = {W[a * 3 + b].x - W[b * 3 + a].x, W[a * 3 + b].y + W[b * 3 + a].y};
                Fm[a * 3 + b] = {-0.5 * d.y, 0.5 * d.x};
            }
        const double tr = (Fm[0].x + Fm[4].x + Fm[8].x) / 3.0;
        Fm[0].x -= tr;
        Fm[4].x -= tr;
        Fm[8].x -= tr;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = Fm[k];
    }
}

}  // namespace

hipError_t launch_force(const Geom &g, const void *gauge64_18, const void *X, const void *Y,
                        void *F, double kappa, const Cplx64 phase[4], int mode, hipStream_t st) {
    const size_t work = (size_t)g.Vh * 2 * 4;
    size_t grid = (work + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(force_kernel, dim3((unsigned)grid), dim3(256), 0, st, g, gauge64_18,
                       (const C *)X, (const C *)Y, (C *)F, kappa, phase[0], phase[1], phase[2],
                       phase[3], mode);
    return hipGetLastError();
}

}  // namespace cola
