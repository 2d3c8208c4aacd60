// Canonical complex128 <-> packed per-parity structure-of-arrays conversion
// for gauge links and spinors, and the SU(3) check that guards the 12-real
// link formats.
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

__device__ __forceinline__ void lex_coords(const Geom &g, uint32_t s, int x[4]) {
    x[0] = (int)(s % (uint32_t)g.L[0]);
    s /= (uint32_t)g.L[0];
    x[1] = (int)(s % (uint32_t)g.L[1]);
    s /= (uint32_t)g.L[1];
    x[2] = (int)(s % (uint32_t)g.L[2]);
    x[3] = (int)(s / (uint32_t)g.L[2]);
}

template <typename T>
__device__ __forceinline__ T to_real(double v) {
    return (T)v;
}

__global__ void pack_gauge_kernel(const Geom g, const cpx<double> *__restrict__ U, void *g64_18,
                                  void *g64_12, void *g32_12, void *g16_12,
                                  unsigned long long *maxdev) {
    const uint32_t V = 2u * (uint32_t)g.Vh;
    double dev = 0.0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < V * 4u;
         t += gridDim.x * blockDim.x) {
        const uint32_t s = t >> 2;
        const int mu = (int)(t & 3u);
        int x[4];
        lex_coords(g, s, x);
        const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
        const uint32_t i = s >> 1;  // Lx even: checkerboard index
        const cpx<double> *u = U + (size_t)t * 9;
        cpx<double> m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = u[k];
        // SU(3) deviation: |U U^H - 1| and |det U - 1|
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                cpx<double> sacc = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) sacc = cmadd(sacc, m[a * 3 + k], cpx<double>{m[b * 3 + k].x, -m[b * 3 + k].y});
                const double re = sacc.x - (a == b ? 1.0 : 0.0);
                dev = fmax(dev, fmax(fabs(re), fabs(sacc.y)));
            }
        const cpx<double> c0 = cmul(m[4], m[8]) - cmul(m[5], m[7]);
        const cpx<double> c1 = cmul(m[5], m[6]) - cmul(m[3], m[8]);
        const cpx<double> c2 = cmul(m[3], m[7]) - cmul(m[4], m[6]);
        cpx<double> det = cmul(m[0], c0);
        det = cmadd(det, m[1], c1);
        det = cmadd(det, m[2], c2);
        dev = fmax(dev, fmax(fabs(det.x - 1.0), fabs(det.y)));
        if (!(dev <= 1e300)) dev = 1e300;  // NaN / Inf
        const size_t S = (size_t)g.S;
        if (g64_18) {
            cpx<double> *o = (cpx<double> *)g64_18 + ((size_t)(p * 4 + mu) * 9) * S + i;
#pragma unroll
            for (int k = 0; k < 9; ++k) o[k * S] = m[k];
        }
        if (g64_12) {
            cpx<double> *o = (cpx<double> *)g64_12 + ((size_t)(p * 4 + mu) * 6) * S + i;
#pragma unroll
            for (int k = 0; k < 6; ++k) o[k * S] = m[k];
        }
        if (g32_12) {
            float4 *o = (float4 *)g32_12 + ((size_t)(p * 4 + mu) * 3) * S + i;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                o[k * S] = make_float4((float)m[2 * k].x, (float)m[2 * k].y, (float)m[2 * k + 1].x,
                                       (float)m[2 * k + 1].y);
        }
        if (g16_12) {
            struct alignas(8) h4 { _Float16 a, b, c, d; };
            h4 *o = (h4 *)g16_12 + ((size_t)(p * 4 + mu) * 3) * S + i;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                h4 v;
                v.a = (_Float16)m[2 * k].x;
                v.b = (_Float16)m[2 * k].y;
                v.c = (_Float16)m[2 * k + 1].x;
                v.d = (_Float16)m[2 * k + 1].y;
                o[k * S] = v;
            }
        }
    }
    // block max, then one atomic max on the (monotone for dev >= 0) bit pattern
    __shared__ double red[256];
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(maxdev, (unsigned long long)__double_as_longlong(red[0]));
}

// One lane per (parity block, checkerboard site, rhs), rhs fastest: the packed side
// (rhs innermost) is written in contiguous runs, and each lane reads its site's 192
// canonical bytes in order.  Only the sites of the packed parities are visited.
template <SpinorFmt F>
__global__ void pack_spinor_kernel(const Geom g, void *dst, const cpx<double> *__restrict__ src,
                                   int nrhs, int parity, size_t block_bytes) {
    using R = typename SpinorT<F>::real;
    const uint32_t V = 2u * (uint32_t)g.Vh;
    const uint32_t per = (uint32_t)g.Vh * (uint32_t)nrhs;  // lanes per parity block
    const uint32_t total = (parity >= 0 ? 1u : 2u) * per;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t blk = t / per;
        const uint32_t e = t - blk * per;
        const uint32_t i = e / (uint32_t)nrhs;
        const uint32_t r = e - i * (uint32_t)nrhs;
        const int p = parity >= 0 ? parity : (int)blk;
        int x[4];
        site_coords(g, i, p, x);
        const uint32_t s = (uint32_t)x[0] +
                           (uint32_t)g.L[0] * ((uint32_t)x[1] + (uint32_t)g.L[1] *
                                               ((uint32_t)x[2] + (uint32_t)g.L[2] * (uint32_t)x[3]));
        const SpinorBlock<F> out((char *)dst + blk * block_bytes, g.S, nrhs);
        cpx<R> v[12];
        const cpx<double> *in = src + ((size_t)r * V + s) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {(R)in[c].x, (R)in[c].y};
        out.store(i, r, v);
    }
}

// The inverse of pack_spinor_kernel; sites of the other parity are left untouched.
template <SpinorFmt F>
__global__ void unpack_spinor_kernel(const Geom g, cpx<double> *__restrict__ dst,
                                     const void *src, int nrhs, int parity, size_t block_bytes) {
    using R = typename SpinorT<F>::real;
    const uint32_t V = 2u * (uint32_t)g.Vh;
    const uint32_t per = (uint32_t)g.Vh * (uint32_t)nrhs;
    const uint32_t total = (parity >= 0 ? 1u : 2u) * per;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += gridDim.x * blockDim.x) {
        const uint32_t blk = t / per;
        const uint32_t e = t - blk * per;
        const uint32_t i = e / (uint32_t)nrhs;
        const uint32_t r = e - i * (uint32_t)nrhs;
        const int p = parity >= 0 ? parity : (int)blk;
        int x[4];
        site_coords(g, i, p, x);
        const uint32_t s = (uint32_t)x[0] +
                           (uint32_t)g.L[0] * ((uint32_t)x[1] + (uint32_t)g.L[1] *
                                               ((uint32_t)x[2] + (uint32_t)g.L[2] * (uint32_t)x[3]));
        const SpinorBlock<F> in((const char *)src + blk * block_bytes, g.S, nrhs);
        cpx<R> v[12];
        in.load(i, r, v);
        cpx<double> *o = dst + ((size_t)r * V + s) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = {(double)v[c].x, (double)v[c].y};
    }
}

int grid_for(size_t work, int block) {
    size_t g = (work + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

size_t spinor_block_bytes(const Geom &g, SpinorFmt f, int nrhs) {
    const size_t SR = (size_t)g.S * nrhs;
    switch (f) {
        case SpinorFmt::F64: return 12 * SR * 16;
        case SpinorFmt::F32: return 12 * SR * 8;
        default: return 12 * SR * 4 + SR * 4;
    }
}

}  // namespace

hipError_t launch_pack_gauge(const Geom &g, const void *U, void *g64_18, void *g64_12,
                             void *g32_12, void *g16_12, unsigned long long *maxdev,
                             hipStream_t st) {
    const size_t work = (size_t)g.Vh * 2 * 4;
    hipLaunchKernelGGL(pack_gauge_kernel, dim3(grid_for(work, 256)), dim3(256), 0, st, g,
                       (const cpx<double> *)U, g64_18, g64_12, g32_12, g16_12, maxdev);
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const Geom &g, SpinorFmt f, void *dst, const void *src, int nrhs,
                              int parity, hipStream_t st) {
    const size_t work = (size_t)g.Vh * 2 * nrhs;
    const size_t bb = spinor_block_bytes(g, f, nrhs);
    const dim3 gr(grid_for(work, 256)), bl(256);
    const cpx<double> *s = (const cpx<double> *)src;
    switch (f) {
        case SpinorFmt::F64: hipLaunchKernelGGL(pack_spinor_kernel<SpinorFmt::F64>, gr, bl, 0, st, g, dst, s, nrhs, parity, bb); break;
        case SpinorFmt::F32: hipLaunchKernelGGL(pack_spinor_kernel<SpinorFmt::F32>, gr, bl, 0, st, g, dst, s, nrhs, parity, bb); break;
        case SpinorFmt::F16: hipLaunchKernelGGL(pack_spinor_kernel<SpinorFmt::F16>, gr, bl, 0, st, g, dst, s, nrhs, parity, bb); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, SpinorFmt f, void *dst, const void *src, int nrhs,
                                int parity, hipStream_t st) {
    const size_t work = (size_t)g.Vh * 2 * nrhs;
    const size_t bb = spinor_block_bytes(g, f, nrhs);
    const dim3 gr(grid_for(work, 256)), bl(256);
    cpx<double> *d = (cpx<double> *)dst;
    switch (f) {
        case SpinorFmt::F64: hipLaunchKernelGGL(unpack_spinor_kernel<SpinorFmt::F64>, gr, bl, 0, st, g, d, src, nrhs, parity, bb); break;
        case SpinorFmt::F32: hipLaunchKernelGGL(unpack_spinor_kernel<SpinorFmt::F32>, gr, bl, 0, st, g, d, src, nrhs, parity, bb); break;
        case SpinorFmt::F16: hipLaunchKernelGGL(unpack_spinor_kernel<SpinorFmt::F16>, gr, bl, 0, st, g, d, src, nrhs, parity, bb); break;
    }
    return hipGetLastError();
}

}  // namespace cola
