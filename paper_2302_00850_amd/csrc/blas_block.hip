// Block kernels for block CG on n right-hand sides held in one packed block:
//   Gram:  G_ab = sum_sites sum_c conj(A_a) B_b              (n x n, FP64 sums)
//   axpy:  X_b += sum_a P_a alpha_ab ;  R_b -= sum_a Q_a alpha_ab
//   xpay:  P'_b = R_b + sum_a P_a beta_ab                    (out of place)
// One lane per (site, column b); the lanes of one site read the same n spinors
// of the site (one cache line per component), so each field is fetched from
// HBM once.  Small matrices are complex FP64, row-major, in device memory.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

size_t bbytes(SpinorFmt f, int S, int R) {
    const size_t SR = (size_t)S * R;
    switch (f) {
        case SpinorFmt::F64: return 12 * SR * 16;
        case SpinorFmt::F32: return 12 * SR * 8;
        default: return 12 * SR * 4 + SR * 4;
    }
}

// component c of (site i, rhs r) in compute precision
template <SpinorFmt F>
__device__ __forceinline__ cpx<typename SpinorT<F>::real> comp(const SpinorBlock<F, true> &v, int c,
                                                              uint32_t i, uint32_t r) {
    const uint32_t e = i * v.nrhs + r;
    const auto h = v.data[c * v.SR + e];
    if constexpr (F == SpinorFmt::F16) {
        const float s = v.norm[e];
        return {s * (float)h.x, s * (float)h.y};
    } else {
        return {h.x, h.y};
    }
}

constexpr int kMaxN = 16;

template <SpinorFmt FA, SpinorFmt FB>
__global__ void __launch_bounds__(256) gram_kernel(const void *A, const void *B, int S, int n,
                                                   int T, Reduce red) {
    extern __shared__ double lds[];
    const SpinorBlock<FA, true> va(A, S, n);
    const SpinorBlock<FB, true> vb(B, S, n);
    double acc[2 * kMaxN];
#pragma unroll
    for (int k = 0; k < 2 * kMaxN; ++k) acc[k] = 0.0;
    const uint32_t total = (uint32_t)S * n;
    const int b = threadIdx.x % n;  // blockDim = T * n, so b is fixed per lane
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t i = t / n;
        for (int c = 0; c < 12; ++c) {
            const auto y = comp(vb, c, i, b);
#pragma unroll
            for (int a = 0; a < kMaxN; ++a) {
                if (a < n) {
                    const auto x = comp(va, c, i, a);
                    // conj(x) * y
                    acc[2 * a] += (double)x.x * y.x + (double)x.y * y.y;
                    acc[2 * a + 1] += (double)x.x * y.y - (double)x.y * y.x;
                }
            }
        }
    }
    // result layout: index (b * n + a) * 2 + {re, im} holds G_ab
    block_sum_to_result<2 * kMaxN>(lds, T, 2 * n * n, threadIdx.x / n, 2 * n * b, 2 * n, acc,
                                   red.partial, red.counter, red.result, blockIdx.x, gridDim.x);
}

// X_b += sum_a P_a al_ab ; R_b -= sum_a Q_a al_ab   (al: n x n complex, row-major)
template <SpinorFmt FX, SpinorFmt FP>
__global__ void __launch_bounds__(256) block_axpy_kernel(void *X, const void *P, void *R,
                                                         const void *Q, const double *al, int S,
                                                         int n) {
    using TX = typename SpinorT<FX>::real;
    const SpinorBlock<FX, true> vx(X, S, n), vr(R, S, n);
    const SpinorBlock<FP, true> vp(P, S, n), vq(Q, S, n);
    const uint32_t total = (uint32_t)S * n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t i = t / n;
        const int b = (int)(t - i * n);
        cpx<TX> xv[12], rv[12];
        vx.load(i, b, xv);
        vr.load(i, b, rv);
        for (int a = 0; a < n; ++a) {
            const cpx<TX> f = {(TX)al[2 * (a * n + b)], (TX)al[2 * (a * n + b) + 1]};
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const auto pa = comp(vp, c, i, a);
                const auto qa = comp(vq, c, i, a);
                xv[c] = cmadd(xv[c], cpx<TX>{(TX)pa.x, (TX)pa.y}, f);
                rv[c] = cmadd(rv[c], cpx<TX>{(TX)-qa.x, (TX)-qa.y}, f);
            }
        }
        vx.store(i, b, xv);
        vr.store(i, b, rv);
    }
}

// Pn_b = R_b + sum_a P_a be_ab
template <SpinorFmt FR, SpinorFmt FP>
__global__ void __launch_bounds__(256) block_xpay_kernel(void *Pn, const void *R, const void *P,
                                                         const double *be, int S, int n) {
    using TP = typename SpinorT<FP>::real;
    const SpinorBlock<FR, true> vr(R, S, n);
    const SpinorBlock<FP, true> vp(P, S, n), vo(Pn, S, n);
    const uint32_t total = (uint32_t)S * n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t i = t / n;
        const int b = (int)(t - i * n);
        cpx<TP> o[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const auto r = comp(vr, c, i, b);
            o[c] = {(TP)r.x, (TP)r.y};
        }
        for (int a = 0; a < n; ++a) {
            const cpx<TP> f = {(TP)be[2 * (a * n + b)], (TP)be[2 * (a * n + b) + 1]};
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const auto pa = comp(vp, c, i, a);
                o[c] = cmadd(o[c], cpx<TP>{(TP)pa.x, (TP)pa.y}, f);
            }
        }
        vo.store(i, b, o);
    }
}

// Z = H^-1 B restricted to the active columns (bit q of act), H Hermitian positive
// semi-definite, read from a Gram result (transposed layout: H_ab at (b n + a) 2), B the
// same way; Z row-major complex.  Cholesky H = L L^H over the active indices in order;
// a pivot below 1e-13 of the largest active diagonal marks a null direction, whose row of
// Z is zero (this deflates linearly dependent search directions); inactive rows and
// columns of Z are zero.  One thread: n <= 16, a few thousand flops.
__global__ void __launch_bounds__(64) block_solve_kernel(const double *Hg, const double *Bg,
                                                         unsigned act, int n, double *Z) {
    __shared__ cpx<double> L[kMaxN * kMaxN];
    __shared__ cpx<double> y[kMaxN];
    __shared__ int ix[kMaxN];
    __shared__ int live[kMaxN];
    if (threadIdx.x != 0) return;
    auto H = [&](int a, int b) { return cpx<double>{Hg[(b * n + a) * 2], Hg[(b * n + a) * 2 + 1]}; };
    auto B = [&](int a, int b) { return cpx<double>{Bg[(b * n + a) * 2], Bg[(b * n + a) * 2 + 1]}; };
    for (int k = 0; k < 2 * n * n; ++k) Z[k] = 0.0;
    int m = 0;
    for (int q = 0; q < n; ++q)
        if (act >> q & 1u) ix[m++] = q;
    if (m == 0) return;
    double dmax = 0.0;
    for (int j = 0; j < m; ++j) dmax = fmax(dmax, H(ix[j], ix[j]).x);
    for (int k = 0; k < m * m; ++k) L[k] = {0.0, 0.0};
    for (int j = 0; j < m; ++j) {
        double d = H(ix[j], ix[j]).x;
        for (int k = 0; k < j; ++k) d -= norm2(L[j * m + k]);
        if (!(d > 1e-13 * dmax)) {
            live[j] = 0;
            continue;
        }
        live[j] = 1;
        const double ljj = sqrt(d);
        L[j * m + j] = {ljj, 0.0};
        for (int i = j + 1; i < m; ++i) {
            cpx<double> s = H(ix[i], ix[j]);
            for (int k = 0; k < j; ++k)
                s = s - cmul(L[i * m + k], cpx<double>{L[j * m + k].x, -L[j * m + k].y});
            L[i * m + j] = {s.x / ljj, s.y / ljj};
        }
    }
    for (int cj = 0; cj < m; ++cj) {
        const int col = ix[cj];
        for (int i = 0; i < m; ++i) {  // L y = b
            if (!live[i]) {
                y[i] = {0.0, 0.0};
                continue;
            }
            cpx<double> s = B(ix[i], col);
            for (int k = 0; k < i; ++k) s = s - cmul(L[i * m + k], y[k]);
            const double l = L[i * m + i].x;
            y[i] = {s.x / l, s.y / l};
        }
        for (int i = m - 1; i >= 0; --i) {  // L^H z = y
            if (!live[i]) {
                y[i] = {0.0, 0.0};
                continue;
            }
            cpx<double> s = y[i];
            for (int k = i + 1; k < m; ++k)
                s = s - cmul(cpx<double>{L[k * m + i].x, -L[k * m + i].y}, y[k]);
            const double l = L[i * m + i].x;
            y[i] = {s.x / l, s.y / l};
        }
        for (int i = 0; i < m; ++i) {
            Z[2 * (ix[i] * n + col)] = y[i].x;
            Z[2 * (ix[i] * n + col) + 1] = y[i].y;
        }
    }
}

struct Shape {
    int T, grid;
};

Shape shape(int S, int n) {
    int T = 1;
    while (T * 2 * n <= 256) T *= 2;
    size_t grid = ((size_t)S * n + (size_t)T * n - 1) / ((size_t)T * n);
    if (grid > 2048) grid = 2048;
    return {T, (int)(grid < 1 ? 1 : grid)};
}

}  // namespace

hipError_t launch_gram(int S, int n, SpinorFmt fa, SpinorFmt fb, const void *A, const void *B,
                       const Reduce &red, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    const Shape sh = shape(S, n);
    const size_t shm = (size_t)sh.T * 2 * n * n * sizeof(double);
    const dim3 g(sh.grid), b(sh.T * n);
#define GRAM(FA, FB) hipLaunchKernelGGL((gram_kernel<FA, FB>), g, b, shm, st, A, B, S, n, sh.T, red)
    if (fa == SpinorFmt::F64 && fb == SpinorFmt::F64) GRAM(SpinorFmt::F64, SpinorFmt::F64);
    else if (fa == SpinorFmt::F32 && fb == SpinorFmt::F32) GRAM(SpinorFmt::F32, SpinorFmt::F32);
    else if (fa == SpinorFmt::F16 && fb == SpinorFmt::F16) GRAM(SpinorFmt::F16, SpinorFmt::F16);
    else return hipErrorInvalidValue;
#undef GRAM
    return hipGetLastError();
}

hipError_t launch_block_axpy(int S, int n, SpinorFmt fx, SpinorFmt fp, void *X, const void *P,
                             void *R, const void *Q, const double *alpha, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    const Shape sh = shape(S, n);
    const dim3 g(sh.grid), b(sh.T * n);
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F16)
        hipLaunchKernelGGL((block_axpy_kernel<SpinorFmt::F32, SpinorFmt::F16>), g, b, 0, st, X, P,
                           R, Q, alpha, S, n);
    else if (fx == SpinorFmt::F32 && fp == SpinorFmt::F32)
        hipLaunchKernelGGL((block_axpy_kernel<SpinorFmt::F32, SpinorFmt::F32>), g, b, 0, st, X, P,
                           R, Q, alpha, S, n);
    else if (fx == SpinorFmt::F64 && fp == SpinorFmt::F64)
        hipLaunchKernelGGL((block_axpy_kernel<SpinorFmt::F64, SpinorFmt::F64>), g, b, 0, st, X, P,
                           R, Q, alpha, S, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_block_solve(const double *H, const double *B, unsigned act, int n, double *Z,
                              hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_solve_kernel, dim3(1), dim3(64), 0, st, H, B, act, n, Z);
    return hipGetLastError();
}

hipError_t launch_block_xpay(int S, int n, SpinorFmt fr, SpinorFmt fp, void *Pn, const void *R,
                             const void *P, const double *beta, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    const Shape sh = shape(S, n);
    const dim3 g(sh.grid), b(sh.T * n);
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F16)
        hipLaunchKernelGGL((block_xpay_kernel<SpinorFmt::F32, SpinorFmt::F16>), g, b, 0, st, Pn, R,
                           P, beta, S, n);
    else if (fr == SpinorFmt::F32 && fp == SpinorFmt::F32)
        hipLaunchKernelGGL((block_xpay_kernel<SpinorFmt::F32, SpinorFmt::F32>), g, b, 0, st, Pn, R,
                           P, beta, S, n);
    else if (fr == SpinorFmt::F64 && fp == SpinorFmt::F64)
        hipLaunchKernelGGL((block_xpay_kernel<SpinorFmt::F64, SpinorFmt::F64>), g, b, 0, st, Pn, R,
                           P, beta, S, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cola
