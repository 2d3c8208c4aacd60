// Vector kernels of the low-eigenmode solver and of deflation: one-rhs FP64 packed
// fields (one parity block, or both blocks of the full lattice), read and written as
// flat arrays of complex doubles (the packed layout is component-major, so every
// field of the same shape lines up element by element).
//
//   eig_dots:     out_j = <V_j, w> = sum conj(V_j) w   for j < k <= kEigChunk
//   eig_lincomb:  out = a out + sum_j c_j V_j         (a = 0: out is not read),
//                 optionally with |out|^2
//   eig_rotate:   x = u x + c q, y = u y + c z, with |x|^2 and <x, y>
//   eig_scale_grad: x *= s, y *= s, g = y - mu x
// (the fused ones spare the launches and passes of a line-search step)
//
// The dot products reduce each lane's partial sums over its wavefront with a fixed
// xor-shuffle butterfly, then over the block's wavefronts in wavefront order, into
// per-block partials; the block-order reduce launch adds those.  Every sum has a fixed
// order, so the results are bitwise reproducible.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

constexpr int kDotThreads = 256;
constexpr int kDotWaves = kDotThreads / 64;

// sum over the 64 lanes of a wavefront; every lane ends with the same bits (IEEE
// addition commutes and each lane's tree has the same pairing)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__global__ void __launch_bounds__(kDotThreads)
    eig_dots_kernel(EigVecs V, int k, const cpx<double> *w, size_t n, double *partial) {
    __shared__ double red[kDotWaves][2 * kEigChunk];
    double acc[2 * kEigChunk];
#pragma unroll
    for (int j = 0; j < 2 * kEigChunk; ++j) acc[j] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const cpx<double> b = w[e];
#pragma unroll
        for (int j = 0; j < kEigChunk; ++j) {
            if (j < k) {
                const cpx<double> a = ((const cpx<double> *)V.v[j])[e];
                acc[2 * j] = fma(a.x, b.x, fma(a.y, b.y, acc[2 * j]));
                acc[2 * j + 1] = fma(a.x, b.y, fma(-a.y, b.x, acc[2 * j + 1]));
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 2 * kEigChunk; ++j) {
        if (j < 2 * k) {
            const double s = wave_sum(acc[j]);
            if (lane == 0) red[wv][j] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * k) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kDotWaves; ++q) s += red[q][threadIdx.x];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

// the block's sums of acc[0..m) (each lane's partial) in wavefront order, into
// partial[j * gridDim.x + blockIdx.x]
template <int M>
__device__ __forceinline__ void block_partials(const double (&acc)[M], double *partial) {
    __shared__ double red[kDotWaves][M];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double s = wave_sum(acc[j]);
        if (lane == 0) red[wv][j] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kDotWaves; ++q) s += red[q][threadIdx.x];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

template <bool NORM>
__global__ void __launch_bounds__(kDotThreads)
    eig_lincomb_kernel(cpx<double> *out, cpx<double> a, EigVecs V, EigCoef c, int k, size_t n,
                       double *partial) {
    double acc[2] = {0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        cpx<double> s = {0.0, 0.0};
        if (a.x != 0.0 || a.y != 0.0) s = cmul(a, out[e]);
#pragma unroll
        for (int j = 0; j < kEigChunk; ++j)
            if (j < k)
                s = cmadd(s, cpx<double>{c.c[j].x, c.c[j].y}, ((const cpx<double> *)V.v[j])[e]);
        out[e] = s;
        if constexpr (NORM) acc[0] = fma(s.x, s.x, fma(s.y, s.y, acc[0]));
    }
    if constexpr (NORM) block_partials<2>(acc, partial);
}

__global__ void __launch_bounds__(kDotThreads)
    eig_rotate_kernel(cpx<double> *x, cpx<double> *y, const cpx<double> *q,
                      const cpx<double> *z, cpx<double> u, cpx<double> c, size_t n,
                      double *partial) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const cpx<double> xv = cmadd(cmul(u, x[e]), c, q[e]);
        const cpx<double> yv = cmadd(cmul(u, y[e]), c, z[e]);
        x[e] = xv;
        y[e] = yv;
        acc[0] = fma(xv.x, xv.x, fma(xv.y, xv.y, acc[0]));
        acc[2] = fma(xv.x, yv.x, fma(xv.y, yv.y, acc[2]));   // Re conj(x) y
        acc[3] = fma(xv.x, yv.y, fma(-xv.y, yv.x, acc[3]));  // Im conj(x) y
    }
    block_partials<4>(acc, partial);
}

__global__ void __launch_bounds__(256)
    eig_scale_grad_kernel(cpx<double> *x, cpx<double> *y, cpx<double> *g, double s, double mu,
                          size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const cpx<double> xv = {s * x[e].x, s * x[e].y};
        const cpx<double> yv = {s * y[e].x, s * y[e].y};
        x[e] = xv;
        y[e] = yv;
        g[e] = {fma(-mu, xv.x, yv.x), fma(-mu, xv.y, yv.y)};
    }
}

int grid_for(size_t n, int cap) {
    size_t g = (n + 255) / 256;
    if (g > (size_t)cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_eig_dots(const EigVecs &V, int k, const void *w, size_t n, double *partial,
                           double *result, hipStream_t st) {
    if (k < 1 || k > kEigChunk) return hipErrorInvalidValue;
    const int grid = grid_for(n, kEigMaxBlocks);
    hipLaunchKernelGGL(eig_dots_kernel, dim3(grid), dim3(kDotThreads), 0, st, V, k,
                       (const cpx<double> *)w, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 2 * k, result, st);
}

hipError_t launch_eig_lincomb(void *out, double are, double aim, const EigVecs &V,
                              const EigCoef &c, int k, size_t n, hipStream_t st,
                              double *partial, double *result) {
    if (k < 0 || k > kEigChunk) return hipErrorInvalidValue;
    if (!result) {
        hipLaunchKernelGGL(eig_lincomb_kernel<false>, dim3(grid_for(n, 8192)), dim3(kDotThreads),
                           0, st, (cpx<double> *)out, cpx<double>{are, aim}, V, c, k, n,
                           nullptr);
        return hipGetLastError();
    }
    const int grid = grid_for(n, kEigMaxBlocks);
    hipLaunchKernelGGL(eig_lincomb_kernel<true>, dim3(grid), dim3(kDotThreads), 0, st,
                       (cpx<double> *)out, cpx<double>{are, aim}, V, c, k, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 2, result, st);
}

hipError_t launch_eig_rotate(void *x, void *y, const void *q, const void *z, Cplx64 u, Cplx64 c,
                             size_t n, double *partial, double *result, hipStream_t st) {
    const int grid = grid_for(n, kEigMaxBlocks);
    hipLaunchKernelGGL(eig_rotate_kernel, dim3(grid), dim3(kDotThreads), 0, st,
                       (cpx<double> *)x, (cpx<double> *)y, (const cpx<double> *)q,
                       (const cpx<double> *)z, cpx<double>{u.x, u.y}, cpx<double>{c.x, c.y}, n,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partial, grid, 4, result, st);
}

hipError_t launch_eig_scale_grad(void *x, void *y, void *g, double s, double mu, size_t n,
                                 hipStream_t st) {
    hipLaunchKernelGGL(eig_scale_grad_kernel, dim3(grid_for(n, 8192)), dim3(256), 0, st,
                       (cpx<double> *)x, (cpx<double> *)y, (cpx<double> *)g, s, mu, n);
    return hipGetLastError();
}

}  // namespace cola
