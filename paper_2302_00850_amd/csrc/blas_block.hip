// Block kernels for block CG on n right-hand sides held in one packed block:
//   Gram:  G_ab = sum_sites sum_c conj(A_a) B_b              (n x n, FP64 sums)
//   axpy:  X_b += sum_a P_a alpha_ab ;  R_b -= sum_a Q_a alpha_ab   (+ optionally R^H R)
//   xpay:  P'_b = R_b + sum_a P_a beta_ab                    (out of place)
// Work comes in units of one component of 16 consecutive sites: in the rhs-innermost
// layout that is 16 n consecutive elements, one per lane, so every load and store of a
// wavefront is contiguous.  A lane keeps column b of the n x n coefficients in registers
// (b = lane mod n, fixed because the block is 16 n lanes); the n columns of its site that
// the mixing needs come from LDS, where each lane put its own element of the unit (two
// buffers, alternating between units, so one barrier per unit suffices).  Small matrices
// are complex FP64, row-major, in device memory.
#include <map>
#include <mutex>
#include <tuple>

#include "device.h"
#include "launch.h"

namespace cola {

namespace {

constexpr int kMaxN = 16;
constexpr int kUnitSites = 16;  // S is a multiple of 64, so units never straddle its end
constexpr int kGramMaxBlocks = 2048;  // Gram partial rows (2 n^2 doubles each) per launch

// element e (= i * n + b) of component c in compute precision T (FP16: times its scale)
template <SpinorFmt F, typename T>
__device__ __forceinline__ cpx<T> load_elem(const SpinorBlock<F, true> &v, int c, uint32_t e) {
    using E = typename SpinorT<F>::elem;
    const E h = bload<E, kCpolNT>(v.comp(c), e * (uint32_t)sizeof(E));
    if constexpr (F == SpinorFmt::F16) {
        const float sc = bload<float, kCpolNT>(v.nrm(), e * 4u);
        return {(T)(sc * (float)h.x), (T)(sc * (float)h.y)};
    } else {
        return {(T)h.x, (T)h.y};
    }
}

template <SpinorFmt F, typename T>
__device__ __forceinline__ void store_elem(const SpinorBlock<F, true> &v, int c, uint32_t e,
                                           cpx<T> z) {
    static_assert(F != SpinorFmt::F16, "element stores are for FP32 / FP64 blocks");
    using E = typename SpinorT<F>::elem;
    bstore<E>(v.comp(c), e * (uint32_t)sizeof(E), E{(typename SpinorT<F>::real)z.x,
                                                   (typename SpinorT<F>::real)z.y});
}

// column b of an n x n row-major complex FP64 matrix, in precision T
template <int N, typename T>
__device__ __forceinline__ void load_column(const double *m, int b, cpx<T> f[N]) {
#pragma unroll
    for (int a = 0; a < N; ++a) f[a] = {(T)m[2 * (a * N + b)], (T)m[2 * (a * N + b) + 1]};
}

// acc_a += conj(x_a) y for the n staged elements x of the lane's site, FP64 products
template <int N, typename T>
__device__ __forceinline__ void gram_acc(const cpx<T> *x, cpx<T> y, double acc[2 * N]) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const cpx<T> xa = x[a];
        acc[2 * a] += (double)xa.x * (double)y.x + (double)xa.y * (double)y.y;
        acc[2 * a + 1] += (double)xa.x * (double)y.y - (double)xa.y * (double)y.x;
    }
}

// The block's Gram partial: lane t holds column b of it (acc[2a], acc[2a + 1] = G_ab) for
// site slot t / n of 16.  Slots s, s + 4, s + 8 are folded into LDS row s mod 4 in that
// order, the lanes of slot s + 12 add that row to their own, and the 4 rows go through
// block_sum_to_result (fixed order throughout: the same sums bit for bit every launch).
// Four rows instead of sixteen keep the LDS of a block at 8 n^2 doubles.
template <int N>
__device__ __forceinline__ void gram_finish(double *lds, double (&acc)[2 * N], int t, int b,
                                            const Reduce &red) {
    constexpr int width = 2 * N * N;
    const int slot = t / N, row = slot & 3, round = slot >> 2;
    double *mine = lds + row * width + 2 * N * b;
    for (int k = t; k < 4 * width; k += blockDim.x) lds[k] = 0.0;
    __syncthreads();
    for (int r = 0; r < 3; ++r) {
        if (round == r) {
#pragma unroll
            for (int k = 0; k < 2 * N; ++k) mine[k] += acc[k];
        }
        __syncthreads();
    }
    if (round == 3) {
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) acc[k] += mine[k];
    }
    __syncthreads();
    block_sum_to_result<2 * N>(lds, 4, width, row, 2 * N * b, round == 3 ? 2 * N : 0, acc,
                               red.partial, red.counter, red.result, blockIdx.x, gridDim.x);
}

// G_ab = sum over sites and components of conj(A_a) B_b.  Lane (unit element) loads its
// B_b and stages its A element; the site's n elements of A then come from LDS.
template <SpinorFmt FA, SpinorFmt FB, int N>
__global__ void __launch_bounds__(256) gram_kernel(const void *A, const void *B, int S,
                                                   Reduce red) {
    using T = typename SpinorT<FA>::real;
    constexpr int W = kUnitSites * N;
    extern __shared__ double lds[];
    __shared__ cpx<T> sa[2][W];
    const SpinorBlock<FA, true> va(A, S, N);
    const SpinorBlock<FB, true> vb(B, S, N);
    const int t = threadIdx.x, b = t % N, s0 = t - b;
    double acc[2 * N];
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) acc[k] = 0.0;
    const uint32_t chunks = (uint32_t)S / kUnitSites, units = 12u * chunks;
    const bool same = A == B;  // A^H A: the lane's B element is its staged A element
    int buf = 0;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x, buf ^= 1) {
        const int c = (int)(u / chunks);
        const uint32_t e = (u - (uint32_t)c * chunks) * W + t;
        const cpx<T> x = load_elem<FA, T>(va, c, e);
        const cpx<T> y = same ? x : load_elem<FB, T>(vb, c, e);
        sa[buf][t] = x;
        __syncthreads();
        gram_acc<N>(&sa[buf][s0], y, acc);
    }
    // result layout: index (b * N + a) * 2 + {re, im} holds G_ab
    gram_finish<N>(lds, acc, t, b, red);
}

//   X_b += sum_a P_a al_ab ;  R_b -= sum_a Q_a al_ab        (al row-major complex FP64)
// GRAM: also G = R^H R of the updated R into red (as gram_kernel), from a second staging
// of the unit (the updated R elements) after a second barrier.
template <SpinorFmt FX, SpinorFmt FP, int N, bool GRAM>
__global__ void __launch_bounds__(256) block_axpy_kernel(void *X, const void *P, void *R,
                                                         const void *Q, const double *al, int S,
                                                         Reduce red) {
    using TX = typename SpinorT<FX>::real;
    constexpr int W = kUnitSites * N;
    extern __shared__ double lds[];
    __shared__ cpx<TX> sp[2][W], sq[2][W];
    __shared__ cpx<TX> sr[GRAM ? 2 : 1][GRAM ? W : 1];
    const SpinorBlock<FX, true> vx(X, S, N), vr(R, S, N);
    const SpinorBlock<FP, true> vp(P, S, N), vq(Q, S, N);
    const int t = threadIdx.x, b = t % N, s0 = t - b;
    cpx<TX> f[N];
    load_column<N>(al, b, f);
    double acc[GRAM ? 2 * N : 1];
#pragma unroll
    for (int k = 0; k < (GRAM ? 2 * N : 1); ++k) acc[k] = 0.0;
    const uint32_t chunks = (uint32_t)S / kUnitSites, units = 12u * chunks;
    int buf = 0;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x, buf ^= 1) {
        const int c = (int)(u / chunks);
        const uint32_t e = (u - (uint32_t)c * chunks) * W + t;
        cpx<TX> x = load_elem<FX, TX>(vx, c, e);
        cpx<TX> r = load_elem<FX, TX>(vr, c, e);
        sp[buf][t] = load_elem<FP, TX>(vp, c, e);
        sq[buf][t] = load_elem<FP, TX>(vq, c, e);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const cpx<TX> pa = sp[buf][s0 + a], qa = sq[buf][s0 + a];
            x = cmadd(x, pa, f[a]);
            r = cmadd(r, cpx<TX>{-qa.x, -qa.y}, f[a]);
        }
        store_elem<FX>(vx, c, e, x);
        store_elem<FX>(vr, c, e, r);
        if constexpr (GRAM) {
            sr[buf][t] = r;
            __syncthreads();
            gram_acc<N>(&sr[buf][s0], r, acc);
        }
    }
    if constexpr (GRAM) gram_finish<N>(lds, acc, t, b, red);
}

// Pn_b = R_b + sum_a P_a be_ab, FP32 / FP64 directions (one lane per unit element)
template <SpinorFmt FR, SpinorFmt FP, int N>
__global__ void __launch_bounds__(256) block_xpay_kernel(void *Pn, const void *R, const void *P,
                                                         const double *be, int S) {
    using TP = typename SpinorT<FP>::real;
    constexpr int W = kUnitSites * N;
    __shared__ cpx<TP> sp[2][W];
    const SpinorBlock<FR, true> vr(R, S, N);
    const SpinorBlock<FP, true> vp(P, S, N), vo(Pn, S, N);
    const int t = threadIdx.x, b = t % N, s0 = t - b;
    cpx<TP> f[N];
    load_column<N>(be, b, f);
    const uint32_t chunks = (uint32_t)S / kUnitSites, units = 12u * chunks;
    int buf = 0;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x, buf ^= 1) {
        const int c = (int)(u / chunks);
        const uint32_t e = (u - (uint32_t)c * chunks) * W + t;
        cpx<TP> o = load_elem<FR, TP>(vr, c, e);
        sp[buf][t] = load_elem<FP, TP>(vp, c, e);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < N; ++a) o = cmadd(o, sp[buf][s0 + a], f[a]);
        store_elem<FP>(vo, c, e, o);
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
        for (int c = 0; c < 12; ++c) o[c] = load_elem<FR, float>(vr, c, t);
        for (int a = 0; a < n; ++a) {
            const cpx<float> f = {(float)be[2 * (a * n + b)], (float)be[2 * (a * n + b) + 1]};
#pragma unroll
            for (int c = 0; c < 12; ++c)
                o[c] = cmadd(o[c], load_elem<SpinorFmt::F16, float>(vp, c, i * n + a), f);
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

// Blocks for a unit kernel (a grid-stride loop over the 12 S / 16 units): as many as are
// resident on the device at once, so that every block takes an equal share of the units
// and no second, partly filled round of blocks trails the first; the reducing kernels
// stay within the Gram partial rows.  Occupancies are cached per (kernel, block, LDS).
int unit_grid(const void *kernel, int block, size_t shm, int S, int ncu, bool reduce) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t>, int> occ_cache;
    int occ = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        const auto key = std::make_tuple(kernel, block, shm);
        auto it = occ_cache.find(key);
        if (it != occ_cache.end()) {
            occ = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, shm) !=
                hipSuccess)
                occ = 1;
            occ_cache[key] = occ;
        }
    }
    const size_t units = (size_t)12 * (S / kUnitSites);
    size_t g = (size_t)(occ < 1 ? 1 : occ) * (size_t)(ncu < 1 ? 1 : ncu);
    if (reduce && g > (size_t)kGramMaxBlocks) g = kGramMaxBlocks;
    if (g > units) g = units;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

#define COLA_BLOCK_N(M)                                                                   \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)

template <SpinorFmt FA, SpinorFmt FB>
hipError_t gram_n(int S, int n, int ncu, const void *A, const void *B, const Reduce &red,
                  hipStream_t st) {
    const size_t shm = (size_t)4 * 2 * n * n * sizeof(double);
    switch (n) {
#define CASE(K)                                                                               \
    case K: {                                                                                 \
        const int grid = unit_grid((const void *)gram_kernel<FA, FB, K>, kUnitSites * K, shm,  \
                                   S, ncu, true);                                             \
        hipLaunchKernelGGL((gram_kernel<FA, FB, K>), dim3(grid), dim3(kUnitSites * K), shm, st, \
                           A, B, S, red);                                                     \
    } break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gram(int S, int n, int ncu, SpinorFmt fa, SpinorFmt fb, const void *A,
                       const void *B, const Reduce &red, hipStream_t st) {
    if (n < 1 || n > kMaxN || fa != fb || S % kUnitSites) return hipErrorInvalidValue;
    switch (fa) {
        case SpinorFmt::F64:
            return gram_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, ncu, A, B, red, st);
        case SpinorFmt::F32:
            return gram_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, ncu, A, B, red, st);
        case SpinorFmt::F16:
            return gram_n<SpinorFmt::F16, SpinorFmt::F16>(S, n, ncu, A, B, red, st);
    }
    return hipErrorInvalidValue;
}

template <SpinorFmt FX, SpinorFmt FP>
hipError_t axpy_n(int S, int n, int ncu, void *X, const void *P, void *R, const void *Q,
                  const double *alpha, const Reduce *gram, hipStream_t st) {
    const Reduce red = gram ? *gram : Reduce{nullptr, nullptr, nullptr};
    const size_t shm = gram ? (size_t)4 * 2 * n * n * sizeof(double) : 0;
    switch (n) {
#define CASE(K)                                                                               \
    case K:                                                                                   \
        if (gram) {                                                                           \
            const int grid = unit_grid((const void *)block_axpy_kernel<FX, FP, K, true>,      \
                                       kUnitSites * K, shm, S, ncu, true);                    \
            hipLaunchKernelGGL((block_axpy_kernel<FX, FP, K, true>), dim3(grid),              \
                               dim3(kUnitSites * K), shm, st, X, P, R, Q, alpha, S, red);     \
        } else {                                                                              \
            const int grid = unit_grid((const void *)block_axpy_kernel<FX, FP, K, false>,     \
                                       kUnitSites * K, 0, S, ncu, false);                     \
            hipLaunchKernelGGL((block_axpy_kernel<FX, FP, K, false>), dim3(grid),             \
                               dim3(kUnitSites * K), 0, st, X, P, R, Q, alpha, S, red);       \
        }                                                                                     \
        break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_block_axpy(int S, int n, int ncu, SpinorFmt fx, SpinorFmt fp, void *X,
                             const void *P, void *R, const void *Q, const double *alpha,
                             const Reduce *gram, hipStream_t st) {
    if (n < 1 || n > kMaxN || S % kUnitSites) return hipErrorInvalidValue;
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F16)
        return axpy_n<SpinorFmt::F32, SpinorFmt::F16>(S, n, ncu, X, P, R, Q, alpha, gram, st);
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F32)
        return axpy_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, ncu, X, P, R, Q, alpha, gram, st);
    if (fx == SpinorFmt::F64 && fp == SpinorFmt::F64)
        return axpy_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, ncu, X, P, R, Q, alpha, gram, st);
    return hipErrorInvalidValue;
}

hipError_t launch_block_solve(const double *H, const double *B, unsigned act, int n, double *Z,
                              hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_solve_kernel, dim3(1), dim3(64), 0, st, H, B, act, n, Z);
    return hipGetLastError();
}

template <SpinorFmt FR, SpinorFmt FP>
hipError_t xpay_n(int S, int n, int ncu, void *Pn, const void *R, const void *P,
                  const double *beta, hipStream_t st) {
    switch (n) {
#define CASE(K)                                                                                \
    case K: {                                                                                  \
        const int grid = unit_grid((const void *)block_xpay_kernel<FR, FP, K>, kUnitSites * K,  \
                                   0, S, ncu, false);                                          \
        hipLaunchKernelGGL((block_xpay_kernel<FR, FP, K>), dim3(grid), dim3(kUnitSites * K), 0, \
                           st, Pn, R, P, beta, S);                                             \
    } break;
        COLA_BLOCK_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_block_xpay(int S, int n, int ncu, SpinorFmt fr, SpinorFmt fp, void *Pn,
                             const void *R, const void *P, const double *beta, hipStream_t st) {
    if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F16) {
        size_t grid = ((size_t)S * n + 255) / 256;
        if (grid > 8192) grid = 8192;
        hipLaunchKernelGGL((block_xpay_h_kernel<SpinorFmt::F32>), dim3(grid), dim3(256), 0, st,
                           Pn, R, P, beta, S, n);
        return hipGetLastError();
    }
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F32)
        return xpay_n<SpinorFmt::F32, SpinorFmt::F32>(S, n, ncu, Pn, R, P, beta, st);
    if (fr == SpinorFmt::F64 && fp == SpinorFmt::F64)
        return xpay_n<SpinorFmt::F64, SpinorFmt::F64>(S, n, ncu, Pn, R, P, beta, st);
    return hipErrorInvalidValue;
}

}  // namespace cola
