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

// The N columns of component c at site i, in compute precision: in the rhs-innermost
// layout they are N consecutive elements (FP16: scaled by the N per-(site, rhs) scales).
template <SpinorFmt F, int N, typename T>
__device__ __forceinline__ void load_row(const SpinorBlock<F, true> &v, int c, uint32_t i,
                                         cpx<T> out[N]) {
    const size_t e = (size_t)c * v.SR + (size_t)i * N;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const auto h = v.data[e + a];
        if constexpr (F == SpinorFmt::F16) {
            const float sc = v.norm[(size_t)i * N + a];
            out[a] = {(T)(sc * (float)h.x), (T)(sc * (float)h.y)};
        } else {
            out[a] = {(T)h.x, (T)h.y};
        }
    }
}

template <SpinorFmt F, int N, typename T>
__device__ __forceinline__ void store_row(const SpinorBlock<F, true> &v, int c, uint32_t i,
                                          const cpx<T> in[N]) {
    static_assert(F != SpinorFmt::F16, "row stores are for FP32 / FP64 blocks");
    const size_t e = (size_t)c * v.SR + (size_t)i * N;
#pragma unroll
    for (int a = 0; a < N; ++a) v.data[e + a] = {(typename SpinorT<F>::real)in[a].x,
                                                (typename SpinorT<F>::real)in[a].y};
}

// G_ab = sum over sites and components of conj(A_a) B_b, FP64 sums.  One lane per (site,
// column b); per component it loads its own B_b and the site's N columns of A (contiguous).
template <SpinorFmt FA, SpinorFmt FB, int N>
__global__ void __launch_bounds__(256) gram_kernel(const void *A, const void *B, int S, int T,
                                                   Reduce red) {
    extern __shared__ double lds[];
    const SpinorBlock<FA, true> va(A, S, N);
    const SpinorBlock<FB, true> vb(B, S, N);
    double acc[2 * N];
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) acc[k] = 0.0;
    const uint32_t total = (uint32_t)S * N;
    const int b = threadIdx.x % N;  // blockDim = T * N, so b is fixed per lane
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t i = t / N;
        for (int c = 0; c < 12; ++c) {
            const auto y = comp(vb, c, i, b);
            cpx<float> x[N];
            if constexpr (FA == SpinorFmt::F64) {
                cpx<double> xd[N];
                load_row<FA, N>(va, c, i, xd);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    acc[2 * a] += xd[a].x * y.x + xd[a].y * y.y;
                    acc[2 * a + 1] += xd[a].x * y.y - xd[a].y * y.x;
                }
            } else {
                load_row<FA, N>(va, c, i, x);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    // conj(x) * y, the products in FP64
                    acc[2 * a] += (double)x[a].x * y.x + (double)x[a].y * y.y;
                    acc[2 * a + 1] += (double)x[a].x * y.y - (double)x[a].y * y.x;
                }
            }
        }
    }
    // result layout: index (b * N + a) * 2 + {re, im} holds G_ab
    block_sum_to_result<2 * N>(lds, T, 2 * N * N, threadIdx.x / N, 2 * N * b, 2 * N, acc,
                               red.partial, red.counter, red.result, blockIdx.x, gridDim.x);
}

// One lane per (component, site): the site's N columns of that component are loaded
// once (consecutive lanes take consecutive sites, so a wavefront reads contiguous
// memory), mixed with the N x N coefficients held in LDS, and stored.
//   X_b += sum_a P_a al_ab ;  R_b -= sum_a Q_a al_ab        (al row-major complex FP64)
template <SpinorFmt FX, SpinorFmt FP, int N>
__global__ void __launch_bounds__(256) block_axpy_kernel(void *X, const void *P, void *R,
                                                         const void *Q, const double *al, int S) {
    using TX = typename SpinorT<FX>::real;
    __shared__ cpx<TX> A[N * N];
    for (int k = threadIdx.x; k < N * N; k += blockDim.x) A[k] = {(TX)al[2 * k], (TX)al[2 * k + 1]};
    __syncthreads();
    const SpinorBlock<FX, true> vx(X, S, N), vr(R, S, N);
    const SpinorBlock<FP, true> vp(P, S, N), vq(Q, S, N);
    const uint32_t total = 12u * (uint32_t)S;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const int c = (int)(t / (uint32_t)S);
        const uint32_t i = t - (uint32_t)c * (uint32_t)S;
        // keeps the coefficient reads from LDS inside the loop: hoisted, the N x N complex
        // coefficients would take 2 N^2 registers
        asm volatile("" ::: "memory");
        cpx<TX> x[N], r[N], p[N], q[N];
        load_row<FX, N>(vx, c, i, x);
        load_row<FX, N>(vr, c, i, r);
        load_row<FP, N>(vp, c, i, p);
        load_row<FP, N>(vq, c, i, q);
#pragma unroll
        for (int b = 0; b < N; ++b) {
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const cpx<TX> f = A[a * N + b];
                x[b] = cmadd(x[b], p[a], f);
                r[b] = cmadd(r[b], cpx<TX>{-q[a].x, -q[a].y}, f);
            }
        }
        store_row<FX, N>(vx, c, i, x);
        store_row<FX, N>(vr, c, i, r);
    }
}

// Pn_b = R_b + sum_a P_a be_ab (one lane per (component, site), as block_axpy_kernel);
// FP32 / FP64 directions

template <SpinorFmt FR, SpinorFmt FP, int N>
__global__ void __launch_bounds__(256) block_xpay_kernel(void *Pn, const void *R, const void *P,
                                                         const double *be, int S) {
    using TP = typename SpinorT<FP>::real;
    __shared__ cpx<TP> B[N * N];
    for (int k = threadIdx.x; k < N * N; k += blockDim.x) B[k] = {(TP)be[2 * k], (TP)be[2 * k + 1]};
    __syncthreads();
    const SpinorBlock<FR, true> vr(R, S, N);
    const SpinorBlock<FP, true> vp(P, S, N), vo(Pn, S, N);
    const uint32_t total = 12u * (uint32_t)S;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const int c = (int)(t / (uint32_t)S);
        const uint32_t i = t - (uint32_t)c * (uint32_t)S;
        asm volatile("" ::: "memory");  // as in block_axpy_kernel
        cpx<TP> r[N], p[N], o[N];
        load_row<FR, N>(vr, c, i, r);
        load_row<FP, N>(vp, c, i, p);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            cpx<TP> s = r[b];
#pragma unroll
            for (int a = 0; a < N; ++a) s = cmadd(s, p[a], B[a * N + b]);
            o[b] = s;
        }
        store_row<FP, N>(vo, c, i, o);
    }
}

// Pn_b = R_b + sum_a P_a be_ab for FP16 directions: one lane per (site, column b), which
// holds all 12 components of its column, as the FP16 store's per-(site, rhs) scale needs
template <SpinorFmt FR>
__global__ void __launch_bounds__(256) block_xpay_h_kernel(void *Pn, const void *R, const void *P,
                                                           const double *be, int S, int n) {
    const SpinorBlock<FR, true> vr(R, S, n);
    const SpinorBlock<SpinorFmt::F16, true> vp(P, S, n), vo(Pn, S, n);
    const uint32_t total = (uint32_t)S * n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t i = t / n;
        const int b = (int)(t - i * n);
        cpx<float> o[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const auto r = comp(vr, c, i, b);
            o[c] = {(float)r.x, (float)r.y};
        }
        for (int a = 0; a < n; ++a) {
            const cpx<float> f = {(float)be[2 * (a * n + b)], (float)be[2 * (a * n + b) + 1]};
#pragma unroll
            for (int c = 0; c < 12; ++c) o[c] = cmadd(o[c], comp(vp, c, i, a), f);
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

#define COLA_BLOCK_N(M)                                                                   \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)

template <SpinorFmt FA, SpinorFmt FB>
hipError_t gram_n(int S, int n, const void *A, const void *B, const Reduce &red, hipStream_t st) {
    const Shape sh = shape(S, n);
    const size_t shm = (size_t)sh.T * 2 * n * n * sizeof(double);
    switch (n) {
#define CASE(K)                                                                               \
    case K:                                                                                   \
        hipLaunchKernelGGL((gram_kernel<FA, FB, K>), dim3(sh.grid), dim3(sh.T * K), shm, st, A, \
                           B, S, sh.T, red);                                                  \
        break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gram(int S, int n, SpinorFmt fa, SpinorFmt fb, const void *A, const void *B,
                       const Reduce &red, hipStream_t st) {
    if (n < 1 || n > kMaxN || fa != fb) return hipErrorInvalidValue;
    switch (fa) {
        case SpinorFmt::F64: return gram_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, A, B, red, st);
        case SpinorFmt::F32: return gram_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, A, B, red, st);
        case SpinorFmt::F16: return gram_n<SpinorFmt::F16, SpinorFmt::F16>(S, n, A, B, red, st);
    }
    return hipErrorInvalidValue;
}

template <SpinorFmt FX, SpinorFmt FP>
hipError_t axpy_n(int S, int n, void *X, const void *P, void *R, const void *Q,
                  const double *alpha, hipStream_t st) {
    size_t grid = ((size_t)12 * S + 255) / 256;
    if (grid > 8192) grid = 8192;
    switch (n) {
#define CASE(K)                                                                               \
    case K:                                                                                   \
        hipLaunchKernelGGL((block_axpy_kernel<FX, FP, K>), dim3(grid), dim3(256), 0, st, X, P, \
                           R, Q, alpha, S);                                                   \
        break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_block_axpy(int S, int n, SpinorFmt fx, SpinorFmt fp, void *X, const void *P,
                             void *R, const void *Q, const double *alpha, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F16)
        return axpy_n<SpinorFmt::F32, SpinorFmt::F16>(S, n, X, P, R, Q, alpha, st);
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F32)
        return axpy_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, X, P, R, Q, alpha, st);
    if (fx == SpinorFmt::F64 && fp == SpinorFmt::F64)
        return axpy_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, X, P, R, Q, alpha, st);
    return hipErrorInvalidValue;
}

hipError_t launch_block_solve(const double *H, const double *B, unsigned act, int n, double *Z,
                              hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_solve_kernel, dim3(1), dim3(64), 0, st, H, B, act, n, Z);
    return hipGetLastError();
}

template <SpinorFmt FR, SpinorFmt FP>
hipError_t xpay_n(int S, int n, void *Pn, const void *R, const void *P, const double *beta,
                  hipStream_t st) {
    size_t grid = ((size_t)12 * S + 255) / 256;
    if (grid > 8192) grid = 8192;
    switch (n) {
#define CASE(K)                                                                                \
    case K:                                                                                    \
        hipLaunchKernelGGL((block_xpay_kernel<FR, FP, K>), dim3(grid), dim3(256), 0, st, Pn, R, \
                           P, beta, S);                                                        \
        break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_block_xpay(int S, int n, SpinorFmt fr, SpinorFmt fp, void *Pn, const void *R,
                             const void *P, const double *beta, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F16) {
        const Shape sh = shape(S, n);
        hipLaunchKernelGGL((block_xpay_h_kernel<SpinorFmt::F32>), dim3(sh.grid), dim3(sh.T * n), 0,
                           st, Pn, R, P, beta, S, n);
        return hipGetLastError();
    }
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F32)
        return xpay_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, Pn, R, P, beta, st);
    if (fr == SpinorFmt::F64 && fp == SpinorFmt::F64)
        return xpay_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, Pn, R, P, beta, st);
    return hipErrorInvalidValue;
}

}  // namespace cola
