// Device-side building blocks: complex arithmetic, site geometry, packed
// spinor/link/clover access and the deterministic block reduction.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace cola {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
    return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
    return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> scale(T s, cpx<T> a) {
    return {s * a.x, s * a.y};
}
// a * b, as explicit fused multiply-adds: the rounding does not depend on how the
// compiler contracts the surrounding code (kernels that must agree bitwise share it)
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
// acc + a * b
template <typename T>
__device__ __forceinline__ cpx<T> cmadd(cpx<T> acc, cpx<T> a, cpx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename T>
__device__ __forceinline__ cpx<T> cjmadd(cpx<T> acc, cpx<T> a, cpx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// a + s*i*b for a real sign s
template <typename T>
__device__ __forceinline__ cpx<T> add_si(cpx<T> a, T s, cpx<T> b) {
    return {fma(-s, b.y, a.x), fma(s, b.x, a.y)};
}
// a + s*b
template <typename T>
__device__ __forceinline__ cpx<T> add_s(cpx<T> a, T s, cpx<T> b) {
    return {fma(s, b.x, a.x), fma(s, b.y, a.y)};
}
template <typename T>
__device__ __forceinline__ T norm2(cpx<T> a) {
    return a.x * a.x + a.y * a.y;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

// XCD-aware work split.  Workgroups are dispatched to the 8 XCDs of the chip
// round-robin (block b runs on XCD b mod 8), each with its own L2.  The nchunks chunks of
// work are cut into one contiguous range per XCD, in proportion to its blocks, so the
// neighbour spinors of a site stay in the L2 of the XCD that computes it.  Block b starts
// at *first and steps by *step (its XCD's block count) up to *end; with G = nchunks every
// block takes one chunk.  The trip count depends on b only.
__device__ __forceinline__ void xcd_range(uint32_t b, uint32_t G, uint32_t nchunks,
                                          uint32_t *first, uint32_t *end, uint32_t *step) {
    const uint32_t q = G >> 3, rem = G & 7u;
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t nbx = q + (x < rem ? 1u : 0u);
    const uint32_t b0 = x * q + (x < rem ? x : rem);  // first logical block of XCD x
    const uint32_t lo = (uint32_t)(((unsigned long long)nchunks * b0) / G);
    const uint32_t hi = (uint32_t)(((unsigned long long)nchunks * (b0 + nbx)) / G);
    *first = lo + k;
    *end = hi;
    *step = nbx;
}

// Coordinates of checkerboard site i of parity p.
__device__ __forceinline__ void site_coords(const Geom &g, uint32_t i, int p, int x[4]) {
    const uint32_t r0 = fdiv(i, g.div_xh);
    const uint32_t xh = i - r0 * (uint32_t)g.Lxh;
    const uint32_t r1 = fdiv(r0, g.div_y);
    x[1] = (int)(r0 - r1 * (uint32_t)g.L[1]);
    const uint32_t r2 = fdiv(r1, g.div_z);
    x[2] = (int)(r1 - r2 * (uint32_t)g.L[2]);
    x[3] = (int)r2;
    x[0] = 2 * (int)xh + ((x[1] + x[2] + x[3] + p) & 1);
}

// Checkerboard index of the neighbour x +- mu (opposite parity).
__device__ __forceinline__ uint32_t nb_fwd(const Geom &g, uint32_t i, const int x[4], int mu) {
    switch (mu) {
        case 0: {
            const uint32_t base = i - (uint32_t)(x[0] >> 1);
            const int xf = x[0] + 1 == g.L[0] ? 0 : x[0] + 1;
            return base + (uint32_t)(xf >> 1);
        }
        case 1: return x[1] == g.L[1] - 1 ? i - (uint32_t)((g.L[1] - 1) * g.s1) : i + g.s1;
        case 2: return x[2] == g.L[2] - 1 ? i - (uint32_t)((g.L[2] - 1) * g.s2) : i + g.s2;
        default: return x[3] == g.L[3] - 1 ? i - (uint32_t)((g.L[3] - 1) * g.s3) : i + g.s3;
    }
}
__device__ __forceinline__ uint32_t nb_bwd(const Geom &g, uint32_t i, const int x[4], int mu) {
    switch (mu) {
        case 0: {
            const uint32_t base = i - (uint32_t)(x[0] >> 1);
            const int xb = x[0] == 0 ? g.L[0] - 1 : x[0] - 1;
            return base + (uint32_t)(xb >> 1);
        }
        case 1: return x[1] == 0 ? i + (uint32_t)((g.L[1] - 1) * g.s1) : i - g.s1;
        case 2: return x[2] == 0 ? i + (uint32_t)((g.L[2] - 1) * g.s2) : i - g.s2;
        default: return x[3] == 0 ? i + (uint32_t)((g.L[3] - 1) * g.s3) : i - g.s3;
    }
}

// ------------------------------------------------------------------ spinors

struct alignas(4) half2s {
    _Float16 x, y;
};

// FP32 -> FP16 (round to nearest even) of two already-rounded FP32 values.  The
// empty asm keeps the compiler from fusing the caller's scaling multiply into a
// mixed-precision conversion (one rounding instead of two) in some instances and not
// in others, which would make the stored halves depend on the launch shape.
__device__ __forceinline__ half2s to_half2(float x, float y) {
    asm volatile("" : "+v"(x), "+v"(y));
    half2s h;
    h.x = (_Float16)x;
    h.y = (_Float16)y;
    return h;
}

template <SpinorFmt F>
struct SpinorT;
template <>
struct SpinorT<SpinorFmt::F64> {
    using real = double;
    using elem = cpx<double>;
};
template <>
struct SpinorT<SpinorFmt::F32> {
    using real = float;
    using elem = cpx<float>;
};
template <>
struct SpinorT<SpinorFmt::F16> {
    using real = float;
    using elem = half2s;
};

// Loads and stores go through buffer resources: one descriptor per component
// array (base = the array, size = its bytes), the per-lane byte offset of the
// site in a VGPR.  Every component of a site then shares one VGPR offset and the
// component base lives in scalar registers, so no per-lane 64-bit address
// arithmetic is spent per load; accesses beyond the descriptor size read zero
// and drop stores.  Arrays handed to one descriptor are below 2^31 bytes
// (checked on the host).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3_t __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// Same for a base known to be uniform across the wavefront: the empty asm makes it
// opaque at each use, so the descriptor is rebuilt next to its loads on the scalar
// unit instead of being hoisted out of the site loop together with dozens of
// others (which overflows the SGPRs).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_u(const void *base, uint32_t bytes) {
    const void *b = base;
    asm volatile("" : "+s"(b));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(b), (short)0, (int)bytes,
                                             0x00020000);
}

// Cache policy of a buffer access (the instruction's cache-policy immediate): 0 is the
// default, kCpolNT sets the nontemporal bit.  Every field store is nontemporal: outputs
// are written once per launch and read by a later launch, and the hint keeps them from
// displacing the neighbour spinors that the hop reuses from L2.  Loads of data used
// once per launch (a site's own spinors in epilogues and vector kernels, clover blocks,
// and the links of one-lane-per-site hops) are nontemporal for the same reason.
constexpr int kCpolNT = 2;

template <typename E, int CP = 0>
__device__ __forceinline__ E bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    E v;
    if constexpr (sizeof(E) == 2) {
        const unsigned short w = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, CP);
        __builtin_memcpy(&v, &w, 2);
    } else if constexpr (sizeof(E) == 4) {
        const unsigned int w = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, CP);
        __builtin_memcpy(&v, &w, 4);
    } else if constexpr (sizeof(E) == 8) {
        const u32x2_t w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, CP);
        __builtin_memcpy(&v, &w, 8);
    } else if constexpr (sizeof(E) == 12) {
        const u32x3_t w = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, 0, CP);
        __builtin_memcpy(&v, &w, 12);
    } else {
        static_assert(sizeof(E) == 16, "16-byte element");
        const u32x4_t w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, CP);
        __builtin_memcpy(&v, &w, 16);
    }
    return v;
}

template <typename E>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, const E &v) {
    if constexpr (sizeof(E) == 4) {
        unsigned int w;
        __builtin_memcpy(&w, &v, 4);
        __builtin_amdgcn_raw_buffer_store_b32(w, r, (int)off, 0, kCpolNT);
    } else if constexpr (sizeof(E) == 8) {
        u32x2_t w;
        __builtin_memcpy(&w, &v, 8);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, kCpolNT);
    } else if constexpr (sizeof(E) == 12) {
        u32x3_t w;
        __builtin_memcpy(&w, &v, 12);
        __builtin_amdgcn_raw_buffer_store_b96(w, r, (int)off, 0, kCpolNT);
    } else {
        static_assert(sizeof(E) == 16, "16-byte element");
        u32x4_t w;
        __builtin_memcpy(&w, &v, 16);
        __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)off, 0, kCpolNT);
    }
}

// View of one parity block of a packed spinor field.  UNI: the block base is the
// same for every lane of a wavefront (true in the hop kernels).
template <SpinorFmt F, bool UNI = false>
struct SpinorBlock {
    using E = typename SpinorT<F>::elem;
    using R = typename SpinorT<F>::real;
    E *data;
    float *norm;     // FP16 only
    uint32_t SR;     // S * nrhs: distance between components (elements)
    uint32_t nrhs;

    __device__ __forceinline__ SpinorBlock(const void *base, int S, int nr)
        : data((E *)base), norm(nullptr), SR((uint32_t)S * nr), nrhs(nr) {
        if (F == SpinorFmt::F16) norm = (float *)(data + 12 * (size_t)SR);
    }

    __device__ __forceinline__ __amdgpu_buffer_rsrc_t comp(int c) const {
        if constexpr (UNI) return buf_u(data + (size_t)c * SR, SR * (uint32_t)sizeof(E));
        return buf(data + (size_t)c * SR, SR * (uint32_t)sizeof(E));
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t nrm() const {
        if constexpr (UNI) return buf_u(norm, SR * 4u);
        return buf(norm, SR * 4u);
    }

    // the 12 components of site i, rhs r, in compute precision
    __device__ __forceinline__ void load(uint32_t i, uint32_t r, cpx<R> v[12]) const {
        R s;
        load_unscaled<kCpolNT>(i, r, v, &s);
        if constexpr (F == SpinorFmt::F16) {
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = {s * v[c].x, s * v[c].y};
        }
    }

    // The 12 components without the FP16 site scale; *scale receives it (1 otherwise).
    template <int CP = 0>
    __device__ __forceinline__ void load_unscaled(uint32_t i, uint32_t r, cpx<R> v[12],
                                                  R *scale) const {
        const uint32_t e = i * nrhs + r;
        const uint32_t off = e * (uint32_t)sizeof(E);
        if constexpr (F == SpinorFmt::F16) {
            *scale = bload<float, CP>(nrm(), e * 4u);
        } else {
            *scale = (R)1;
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const E h = bload<E, CP>(comp(c), off);
            v[c] = {(R)h.x, (R)h.y};
        }
    }

    // FP16 only: the raw packed halves of site i, rhs r and the site scale.
    template <typename H2>
    __device__ __forceinline__ void load_raw_h2(uint32_t i, uint32_t r, H2 v[12],
                                                float *scale) const {
        static_assert(F == SpinorFmt::F16, "packed halves exist for FP16 blocks only");
        const uint32_t e = i * nrhs + r;
        const uint32_t off = e * (uint32_t)sizeof(E);
        *scale = bload<float>(nrm(), e * 4u);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = bload<H2>(comp(c), off);
    }

    // FP16 only: raw halves and site scales of the N consecutive right-hand sides
    // r0 .. r0+N-1 of site i (r0 and the block's rhs count multiples of N), one
    // N x 4-byte load per component.
    template <int N, typename H2>
    __device__ __forceinline__ void load_raw_h2_group(uint32_t i, uint32_t r0, H2 v[N][12],
                                                      float scale[N]) const {
        static_assert(F == SpinorFmt::F16, "packed halves exist for FP16 blocks only");
        struct G { H2 x[N]; };
        struct FS { float x[N]; };
        const uint32_t off = (i * nrhs + r0) * 4u;
        const FS f = bload<FS>(nrm(), off);
#pragma unroll
        for (int r = 0; r < N; ++r) scale[r] = f.x[r];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const G w = bload<G>(comp(c), off);
#pragma unroll
            for (int r = 0; r < N; ++r) v[r][c] = w.x[r];
        }
    }

    // FP16 only: store N consecutive right-hand sides of site i (as load_raw_h2_group);
    // with keep, v is replaced by the values actually stored.
    template <int N>
    __device__ __forceinline__ void store_group(uint32_t i, uint32_t r0, cpx<float> v[N][12],
                                                bool keep) const {
        static_assert(F == SpinorFmt::F16, "grouped stores are for FP16 blocks");
        struct G { half2s x[N]; };
        struct FS { float x[N]; };
        const uint32_t off = (i * nrhs + r0) * 4u;
        G w[12];
        FS f;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            float m = 0.f;
#pragma unroll
            for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[r][c].x), fabsf(v[r][c].y)));
            if (!(m >= 1e-30f) && m == m) m = 0.f;  // as in store()
            const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const half2s h = to_half2(v[r][c].x * inv, v[r][c].y * inv);
                w[c].x[r] = h;
                if (keep) v[r][c] = {m * (float)h.x, m * (float)h.y};
            }
            f.x[r] = m;
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) bstore<G>(comp(c), off, w[c]);
        bstore<FS>(nrm(), off, f);
    }

    // Store; v is replaced by the values actually stored (FP16 rounding).
    __device__ __forceinline__ void store(uint32_t i, uint32_t r, cpx<R> v[12]) const {
        const uint32_t e = i * nrhs + r;
        const uint32_t off = e * (uint32_t)sizeof(E);
        if constexpr (F == SpinorFmt::F16) {
            float m = 0.f;
#pragma unroll
            for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
            // a site whose largest entry is below 1e-30 is stored as zero: 1/m would
            // overflow for FP32 denormals (point-source propagators decay that far)
            if (!(m >= 1e-30f) && m == m) m = 0.f;
            const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const half2s h = to_half2(v[c].x * inv, v[c].y * inv);
                bstore<E>(comp(c), off, h);
                v[c] = {m * (float)h.x, m * (float)h.y};
            }
            bstore<float>(nrm(), e * 4u, m);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) bstore<E>(comp(c), off, E{v[c].x, v[c].y});
        }
    }
};

// ------------------------------------------------------------------- links

template <LinkFmt F>
struct LinkT;
template <>
struct LinkT<LinkFmt::F64_18> {
    using real = double;
    struct alignas(16) chunk { double a, b; };
};
template <>
struct LinkT<LinkFmt::F64_12> {
    using real = double;
    struct alignas(16) chunk { double a, b; };
};
template <>
struct LinkT<LinkFmt::F32_12> {
    using real = float;
    struct alignas(16) chunk { float a, b, c, d; };
};
template <>
struct LinkT<LinkFmt::F16_12> {
    using real = float;
    struct alignas(8) chunk { _Float16 a, b, c, d; };
};

// row 2 = conj(row 0 x row 1) of a 12-real link: with a = row 0, b = row 1 and
// (k, k1, k2) cyclic, row2_k = conj(a_k1 b_k2 - a_k2 b_k1).  Written as explicit fused
// multiply-adds, so every caller rounds the same way.
template <typename T>
__device__ __forceinline__ void rebuild_row2(cpx<T> u[3][3]) {
    const cpx<T> *a = u[0], *b = u[1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const T re = fma(a[k1].x, b[k2].x,
                         fma(-a[k1].y, b[k2].y, fma(-a[k2].x, b[k1].x, a[k2].y * b[k1].y)));
        const T im = fma(a[k1].x, b[k2].y,
                         fma(a[k1].y, b[k2].x, fma(-a[k2].x, b[k1].y, -(a[k2].y * b[k1].x))));
        u[2][k] = {re, -im};
    }
}

// Load U_mu at checkerboard site i of parity p; row 2 rebuilt as conj(row0 x row1)
// for the 12-real formats.
// UNI: parity p is the same for every lane of the wavefront.  CP: cache policy.
template <LinkFmt F, typename T, bool UNI = true, int CP = 0>
__device__ __forceinline__ void load_link(const void *gauge, int S, int p, int mu, uint32_t i,
                                          cpx<T> u[3][3]) {
    using CH = typename LinkT<F>::chunk;
    const auto buf_u = [](const void *b, uint32_t n) {
        if constexpr (UNI) return ::cola::buf_u(b, n);
        return ::cola::buf(b, n);
    };
    constexpr int N = link_chunks(F);
    const CH *base = (const CH *)gauge + ((size_t)(p * 4 + mu) * N) * (size_t)S;  // uniform
    const uint32_t off = i * (uint32_t)sizeof(CH);
    if constexpr (F == LinkFmt::F64_18) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const CH c = bload<CH, CP>(buf_u(base + (size_t)k * S, (uint32_t)S * sizeof(CH)), off);
            u[k / 3][k % 3] = {(T)c.a, (T)c.b};
        }
        return;
    } else if constexpr (F == LinkFmt::F64_12) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const CH c = bload<CH, CP>(buf_u(base + (size_t)k * S, (uint32_t)S * sizeof(CH)), off);
            u[k / 3][k % 3] = {(T)c.a, (T)c.b};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const CH c = bload<CH, CP>(buf_u(base + (size_t)k * S, (uint32_t)S * sizeof(CH)), off);
            u[(2 * k) / 3][(2 * k) % 3] = {(T)c.a, (T)c.b};
            u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {(T)c.c, (T)c.d};
        }
    }
    if constexpr (F != LinkFmt::F64_18) rebuild_row2(u);
}

// w = U h
template <typename T>
__device__ __forceinline__ void su3_mul(const cpx<T> u[3][3], const cpx<T> h[3], cpx<T> w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> s = cmul(u[a][0], h[0]);
        s = cmadd(s, u[a][1], h[1]);
        s = cmadd(s, u[a][2], h[2]);
        w[a] = s;
    }
}
// w = U^H h
template <typename T>
__device__ __forceinline__ void su3_dag_mul(const cpx<T> u[3][3], const cpx<T> h[3],
                                            cpx<T> w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> s = {(T)0, (T)0};
        s = cjmadd(s, u[0][a], h[0]);
        s = cjmadd(s, u[1][a], h[1]);
        s = cjmadd(s, u[2][a], h[2]);
        w[a] = s;
    }
}

// ------------------------------------------------------- spin projection

// Spin projection with (1 + sg g_mu) in the chiral basis, sg = +-1:
//   mu=x: h0 = p0 + sg i p3, h1 = p1 + sg i p2; lower: s2 += -sg i W1, s3 += -sg i W0
//   mu=y: h0 = p0 - sg p3,   h1 = p1 + sg p2;   lower: s2 +=  sg W1,   s3 += -sg W0
//   mu=z: h0 = p0 + sg i p2, h1 = p1 - sg i p3; lower: s2 += -sg i W0, s3 +=  sg i W1
//   mu=t: h0 = p0 + sg p2,   h1 = p1 + sg p3;   lower: s2 +=  sg W0,   s3 +=  sg W1
// where the upper spins receive W0 and W1.  expand_add(project(psi)) with W = h
// is (1 + sg g_mu) psi.
template <typename T>
__device__ __forceinline__ void project(int mu, T sg, const cpx<T> p[12], cpx<T> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        switch (mu) {
            case 0: h[c] = add_si(p0, sg, p3); h[3 + c] = add_si(p1, sg, p2); break;
            case 1: h[c] = add_s(p0, -sg, p3); h[3 + c] = add_s(p1, sg, p2); break;
            case 2: h[c] = add_si(p0, sg, p2); h[3 + c] = add_si(p1, -sg, p3); break;
            default: h[c] = add_s(p0, sg, p2); h[3 + c] = add_s(p1, sg, p3); break;
        }
    }
}

template <typename T>
__device__ __forceinline__ void expand_add(int mu, T sg, const cpx<T> w[6], cpx<T> acc[12],
                                           T s = (T)1) {
    // acc += s * (1 + sg g_mu) expansion of (w0, w1); s is a real boundary phase
    const T ts = sg * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> w0 = w[c], w1 = w[3 + c];
        acc[c] = add_s(acc[c], s, w0);
        acc[3 + c] = add_s(acc[3 + c], s, w1);
        switch (mu) {
            case 0:
                acc[6 + c] = add_si(acc[6 + c], -ts, w1);
                acc[9 + c] = add_si(acc[9 + c], -ts, w0);
                break;
            case 1:
                acc[6 + c] = add_s(acc[6 + c], ts, w1);
                acc[9 + c] = add_s(acc[9 + c], -ts, w0);
                break;
            case 2:
                acc[6 + c] = add_si(acc[6 + c], -ts, w0);
                acc[9 + c] = add_si(acc[9 + c], ts, w1);
                break;
            default:
                acc[6 + c] = add_s(acc[6 + c], ts, w0);
                acc[9 + c] = add_s(acc[9 + c], ts, w1);
                break;
        }
    }
}

// ------------------------------------------------ FP16 packed path (dot2 products)

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// a + s b and a + s i b on packed (re, im) halves; one v_pk_fma_f16 each
__device__ __forceinline__ h2 add_s_h2(h2 a, _Float16 s, h2 b) { return a + h2{s, s} * b; }
__device__ __forceinline__ h2 add_si_h2(h2 a, _Float16 s, h2 b) {
    return a + h2{s, s} * h2{-b.y, b.x};
}

// Spin projection (1 + sg g_mu) of a spinor held as packed halves (same table as project).
__device__ __forceinline__ void project_h2(int mu, _Float16 sg, const h2 p[12], h2 h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2 p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        switch (mu) {
            case 0: h[c] = add_si_h2(p0, sg, p3); h[3 + c] = add_si_h2(p1, sg, p2); break;
            case 1: h[c] = add_s_h2(p0, -sg, p3); h[3 + c] = add_s_h2(p1, sg, p2); break;
            case 2: h[c] = add_si_h2(p0, sg, p2); h[3 + c] = add_si_h2(p1, -sg, p3); break;
            default: h[c] = add_s_h2(p0, sg, p2); h[3 + c] = add_s_h2(p1, sg, p3); break;
        }
    }
}

// FP16 link prepared as dot2 operand pairs (one v_dot2 per real output term: the
// FP16 x FP16 products are exact and summed in FP32).  For w = V h:
//   V = U:   re = sum dot(A_ab, h_b) with A = (u.x, -u.y);  im: B = (u.y, u.x)
//   V = U^H: A_ab = u_ba;                                   B_ab = (-u_ba.y, u_ba.x)
struct LinkH2 {
    h2 A[3][3];
    h2 B[3][3];
};

__device__ __forceinline__ float dot2(h2 a, h2 b, float c) {
    return __builtin_amdgcn_fdot2(a, b, c, false);
}

// Rows 0 and 1 of L.u given: row 2 = conj(row0 x row1) from dot2 products of the stored
// halves, rounded once to FP16.  With a = row 0, b = row 1 and (k, k1, k2) cyclic,
//   re row2_k =  Re(a_k1 b_k2) - Re(a_k2 b_k1) = dot(a_k1, (b.x, -b.y)_k2) + dot(a_k2, (-b.x, b.y)_k1)
//   im row2_k = -Im(a_k1 b_k2) + Im(a_k2 b_k1) = dot(a_k1, (-b.y, -b.x)_k2) + dot(a_k2, (b.y, b.x)_k1)
__device__ __forceinline__ void link_h2_row2(h2 u[3][3]) {
    h2 bc[3], bn[3], bs[3], bsn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const h2 v = u[1][k];
        bc[k] = h2{v.x, -v.y};
        bn[k] = h2{-v.x, v.y};
        bs[k] = h2{v.y, v.x};
        bsn[k] = h2{-v.y, -v.x};
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const float re = dot2(u[0][k2], bn[k1], dot2(u[0][k1], bc[k2], 0.f));
        const float im = dot2(u[0][k2], bs[k1], dot2(u[0][k1], bsn[k2], 0.f));
        u[2][k] = h2{(_Float16)re, (_Float16)im};
    }
}

// The dot2 operands of V = U (DAG false) or V = U^H (DAG true) from the full link u.
template <bool DAG>
__device__ __forceinline__ void link_h2_prepare(const h2 u[3][3], LinkH2 &L) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (DAG) {
                const h2 v = u[b][a];
                L.A[a][b] = v;
                L.B[a][b] = h2{-v.y, v.x};
            } else {
                const h2 v = u[a][b];
                L.A[a][b] = h2{v.x, -v.y};
                L.B[a][b] = h2{v.y, v.x};
            }
        }
}

// Load U_mu at checkerboard site i of parity p (rows 0 and 1 stored, row 2 rebuilt) as
// the dot2 operands of V = U (DAG false) or V = U^H (DAG true).
template <bool DAG>
__device__ __forceinline__ void load_link_h2(const void *gauge, int S, int p, int mu, uint32_t i,
                                             LinkH2 &L) {
    using CH = LinkT<LinkFmt::F16_12>::chunk;
    const CH *base = (const CH *)gauge + ((size_t)(p * 4 + mu) * 3) * (size_t)S;
    const uint32_t off = i * (uint32_t)sizeof(CH);
    h2 u[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const CH c = bload<CH>(buf_u(base + (size_t)k * S, (uint32_t)S * sizeof(CH)), off);
        u[(2 * k) / 3][(2 * k) % 3] = h2{c.a, c.b};
        u[(2 * k + 1) / 3][(2 * k + 1) % 3] = h2{c.c, c.d};
    }
    link_h2_row2(u);
    link_h2_prepare<DAG>(u, L);
}

// w = V h for one colour vector h (V as prepared in L): three dot2 per real output.
__device__ __forceinline__ void mul_h2(const LinkH2 &L, const h2 h[3], cpx<float> w[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float re = dot2(L.A[a][0], h[0], 0.f);
        float im = dot2(L.B[a][0], h[0], 0.f);
        re = dot2(L.A[a][1], h[1], re);
        im = dot2(L.B[a][1], h[1], im);
        re = dot2(L.A[a][2], h[2], re);
        im = dot2(L.B[a][2], h[2], im);
        w[a] = {re, im};
    }
}

// ------------------------------------------- links staged by the lanes of a site

// In the multi-rhs hop the lanes of one site can split its eight links between them:
// lane j < 8 loads and rebuilds link j (mu = j / 2, backward for odd j) once and leaves
// it in LDS for all the site's lanes.  The direction is then a per-lane value, so these
// helpers take it at run time without divergent branches.  A staged link is 18 words:
// FP16 links as their dot2 operands (A then B, of U or U^H), FP32 links as the nine
// complex entries of U.
constexpr int kStageWords = 20;                  // per link (18 used, 16-byte multiple)
constexpr int kStageSite = 8 * kStageWords + 4;  // per site (padding spreads LDS banks)

// backward neighbour x - mu for a run-time mu: every candidate, then a select
__device__ __forceinline__ uint32_t nb_bwd_rt(const Geom &g, uint32_t i, const int x[4], int mu) {
    const uint32_t base = i - (uint32_t)(x[0] >> 1);
    const int xb = x[0] == 0 ? g.L[0] - 1 : x[0] - 1;
    const uint32_t n0 = base + (uint32_t)(xb >> 1);
    const uint32_t n1 = x[1] == 0 ? i + (uint32_t)((g.L[1] - 1) * g.s1) : i - g.s1;
    const uint32_t n2 = x[2] == 0 ? i + (uint32_t)((g.L[2] - 1) * g.s2) : i - g.s2;
    const uint32_t n3 = x[3] == 0 ? i + (uint32_t)((g.L[3] - 1) * g.s3) : i - g.s3;
    const uint32_t a = mu == 0 ? n0 : n1, b = mu == 2 ? n2 : n3;
    return mu < 2 ? a : b;
}

// chunk k of U_mu at (p, i) for run-time p and mu: one descriptor over the whole packed
// gauge field (below 2^31 bytes, checked on the host), per-lane byte offset
template <LinkFmt F>
__device__ __forceinline__ typename LinkT<F>::chunk load_chunk_rt(const void *gauge, int S, int p,
                                                                  int mu, int k, uint32_t i) {
    using CH = typename LinkT<F>::chunk;
    constexpr int N = link_chunks(F);
    const uint32_t bytes = 8u * (uint32_t)N * (uint32_t)S * (uint32_t)sizeof(CH);
    const uint32_t off =
        ((uint32_t)((p * 4 + mu) * N + k) * (uint32_t)S + i) * (uint32_t)sizeof(CH);
    return bload<CH>(buf_u(gauge, bytes), off);
}

// Stage link (mu, back) of output site i (backward: U_mu at neighbour n, parity 1 - p).
template <LinkFmt F>
__device__ __forceinline__ void stage_link(const void *gauge, int S, int p, int mu, bool back,
                                           uint32_t i, uint32_t n, uint32_t *dst) {
    using CH = typename LinkT<F>::chunk;
    static_assert(F == LinkFmt::F16_12 || F == LinkFmt::F32_12, "12-real links only");
    const int pl = back ? 1 - p : p;
    const uint32_t il = back ? n : i;
    uint32_t w[kStageWords];
    if constexpr (F == LinkFmt::F16_12) {
        h2 u[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const CH c = load_chunk_rt<F>(gauge, S, pl, mu, k, il);
            u[(2 * k) / 3][(2 * k) % 3] = h2{c.a, c.b};
            u[(2 * k + 1) / 3][(2 * k + 1) % 3] = h2{c.c, c.d};
        }
        link_h2_row2(u);
        LinkH2 Lf, Lb;
        link_h2_prepare<false>(u, Lf);
        link_h2_prepare<true>(u, Lb);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const h2 A = back ? Lb.A[a][b] : Lf.A[a][b];
                const h2 B = back ? Lb.B[a][b] : Lf.B[a][b];
                __builtin_memcpy(&w[3 * a + b], &A, 4);
                __builtin_memcpy(&w[9 + 3 * a + b], &B, 4);
            }
    } else {
        cpx<float> u[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const CH c = load_chunk_rt<F>(gauge, S, pl, mu, k, il);
            u[(2 * k) / 3][(2 * k) % 3] = {c.a, c.b};
            u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {c.c, c.d};
        }
        rebuild_row2(u);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                __builtin_memcpy(&w[2 * (3 * a + b)], &u[a][b].x, 4);
                __builtin_memcpy(&w[2 * (3 * a + b) + 1], &u[a][b].y, 4);
            }
    }
    w[18] = w[19] = 0u;
#pragma unroll
    for (int k = 0; k < kStageWords; k += 4)
        *(u32x4_t *)(dst + k) = u32x4_t{w[k], w[k + 1], w[k + 2], w[k + 3]};
}

// read back a staged link
__device__ __forceinline__ void read_staged(const uint32_t *src, LinkH2 &L) {
    uint32_t w[kStageWords];
#pragma unroll
    for (int k = 0; k < kStageWords; k += 4) {
        const u32x4_t v = *(const u32x4_t *)(src + k);
        w[k] = v.x, w[k + 1] = v.y, w[k + 2] = v.z, w[k + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        __builtin_memcpy(&L.A[k / 3][k % 3], &w[k], 4);
        __builtin_memcpy(&L.B[k / 3][k % 3], &w[9 + k], 4);
    }
}
__device__ __forceinline__ void read_staged(const uint32_t *src, cpx<float> u[3][3]) {
    uint32_t w[kStageWords];
#pragma unroll
    for (int k = 0; k < kStageWords; k += 4) {
        const u32x4_t v = *(const u32x4_t *)(src + k);
        w[k] = v.x, w[k + 1] = v.y, w[k + 2] = v.z, w[k + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        __builtin_memcpy(&u[k / 3][k % 3].x, &w[2 * k], 4);
        __builtin_memcpy(&u[k / 3][k % 3].y, &w[2 * k + 1], 4);
    }
}

// ------------------------------------------------------------------ clover

// out = C in, C = two Hermitian 6x6 chiral blocks (spins {0,1} and {2,3}).
template <typename CR, typename T>
__device__ __forceinline__ void clover_apply(const void *clov, int S, int p, uint32_t i,
                                             const cpx<T> in[12], cpx<T> out[12]) {
    struct pair { CR a, b; };
    const pair *base = (const pair *)clov + (size_t)(p * 36) * S;  // uniform
    const uint32_t off = i * (uint32_t)sizeof(pair);
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const pair *q = base + (size_t)(blk * 18) * S;
        T d[6];
        cpx<T> o[15];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const pair v =
                bload<pair, kCpolNT>(buf_u(q + (size_t)k * S, (uint32_t)S * sizeof(pair)), off);
            d[2 * k] = (T)v.a;
            d[2 * k + 1] = (T)v.b;
        }
#pragma unroll
        for (int k = 0; k < 15; ++k) {
            const pair v =
                bload<pair, kCpolNT>(buf_u(q + (size_t)(3 + k) * S, (uint32_t)S * sizeof(pair)), off);
            o[k] = {(T)v.a, (T)v.b};
        }
        const cpx<T> *v = in + 6 * blk;
        cpx<T> *y = out + 6 * blk;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            cpx<T> s = scale(d[r], v[r]);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                if (c < r) s = cmadd(s, o[r * (r - 1) / 2 + c], v[c]);
                if (c > r) s = cjmadd(s, o[c * (c - 1) / 2 + r], v[c]);
            }
            y[r] = s;
        }
    }
}

// out = C in from a site's clover block staged in LDS: pair m (0..35, as in memory, the
// second chiral block from m = 18) at c[2m], c[2m + 1].  The same arithmetic, in the same
// order, as clover_apply.
constexpr int kClovStage = 76;  // floats per staged site (72 used; the padding spreads banks)

template <typename T>
__device__ __forceinline__ void clover_apply_lds(const float *c, const cpx<T> in[12],
                                                 cpx<T> out[12]) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const float *q = c + 36 * blk;
        float w[36];
#pragma unroll
        for (int k = 0; k < 36; k += 4) {
            const float4 v = *(const float4 *)(q + k);
            w[k] = v.x;
            w[k + 1] = v.y;
            w[k + 2] = v.z;
            w[k + 3] = v.w;
        }
        T d[6];
        cpx<T> o[15];
#pragma unroll
        for (int k = 0; k < 6; ++k) d[k] = (T)w[k];
#pragma unroll
        for (int k = 0; k < 15; ++k) o[k] = {(T)w[6 + 2 * k], (T)w[7 + 2 * k]};
        const cpx<T> *v = in + 6 * blk;
        cpx<T> *y = out + 6 * blk;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            cpx<T> s = scale(d[r], v[r]);
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) {
                if (cc < r) s = cmadd(s, o[r * (r - 1) / 2 + cc], v[cc]);
                if (cc > r) s = cjmadd(s, o[cc * (cc - 1) / 2 + r], v[cc]);
            }
            y[r] = s;
        }
    }
}

// Stage pair m of the FP32 clover block of site i (parity p) into c[2m], c[2m + 1].
__device__ __forceinline__ void stage_clover_pair(const void *clov, int S, int p, uint32_t i,
                                                  int m, float *c) {
    struct pair { float a, b; };
    const pair *base = (const pair *)clov + (size_t)(p * 36 + m) * S;
    const pair v = bload<pair, kCpolNT>(buf(base, (uint32_t)S * sizeof(pair)), i * 8u);
    c[2 * m] = v.a;
    c[2 * m + 1] = v.b;
}

// ---------------------------------------------------------------- reduction

// Per-block part of a two-kernel reduction: the lanes' values v[0..n) for columns q0..
// q0 + n are summed over the block into partial[q * nblocks + bid] (column-major, so the
// reduction reads each column contiguously).  Lane t owns columns (t mod g) n .. + n,
// g = width / n (the callers' layout: slot t / g, q0 = (t mod g) n), so lanes t and
// t + g m share columns.  Within a wavefront those lanes are summed by shuffles (an xor
// butterfly when g is a power of two and the wavefront is whole, else a chain in lane
// order), then the wavefronts' sums in wavefront order through LDS (red holds T * width
// doubles, T = blockDim / g).  A following reduce_partials launch adds the blocks'
// partials in block order; the kernel boundary orders the writes, so blocks need no
// fence or ticket (device-scope fences write back the XCD's L2 on this chip: with tens
// of thousands of blocks they cost more than the kernel).  Every sum has a fixed order.
template <int NV>
__device__ void block_sum_to_partial(double *red, int T, int width, int slot, int q0, int n,
                                     const double (&v)[NV], double *partial, uint32_t bid,
                                     uint32_t nblocks) {
    (void)T;
    (void)slot;
    (void)q0;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int g = width / n;
    const int lane = tid & 63, wave = tid >> 6, nwaves = (nt + 63) >> 6;
    const int live = min(64, nt - 64 * wave);  // lanes of this wavefront
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = v[k];
    if ((g & (g - 1)) == 0 && live == 64) {
        for (int off = 32; off >= g; off >>= 1) {
#pragma unroll
            for (int k = 0; k < NV; ++k) s[k] += __shfl_xor(s[k], off);
        }
    } else {
        for (int m = g; m < 64; m += g) {
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const double o = __shfl(v[k], (lane + m) & 63);
                if (lane + m < live) s[k] += o;
            }
        }
    }
    for (int k = tid; k < nwaves * width; k += nt) red[k] = 0.0;
    __syncthreads();
    if (lane < g && lane < live) {
        const int j = tid % g;
#pragma unroll
        for (int k = 0; k < NV; ++k)  // constant indices keep s in registers
            if (k < n) red[wave * width + j * n + k] = s[k];
    }
    __syncthreads();
    for (int q = tid; q < width; q += nt) {
        double a = red[q];
        for (int w = 1; w < nwaves; ++w) a += red[w * width + q];
        partial[(size_t)q * nblocks + bid] = a;
    }
}

// Deterministic per-block reduction: the lanes' values v[0..n) for columns q0.. of
// slot `slot` are summed over the block (LDS tree over the T slots of red, which holds
// T * width doubles) into partial[bid][q].  The last block of each group of kRedGroup
// blocks (atomic ticket) adds its group's partials in block order; the last group to
// finish adds the group sums in group order into result[q].  Every sum has a fixed
// order whatever the timing, and each stage adds at most kRedGroup terms per column.
// The tickets are re-armed to zero.
template <int NV>
__device__ void block_sum_to_result(double *red, int T, int width, int slot, int q0, int n,
                                    const double (&v)[NV], double *partial, unsigned *counter,
                                    double *result, uint32_t bid, uint32_t nblocks) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int k = tid; k < T * width; k += nt) red[k] = 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k)  // constant indices keep v in registers
        if (k < n) red[slot * width + q0 + k] = v[k];
    __syncthreads();
    for (int w = T >> 1; w > 0; w >>= 1) {
        for (int k = tid; k < w * width; k += nt) red[k] += red[k + w * width];
        __syncthreads();
    }
    for (int k = tid; k < width; k += nt) partial[(size_t)bid * width + k] = red[k];

    const uint32_t group = bid / (uint32_t)kRedGroup;
    const uint32_t ngroups = (nblocks + kRedGroup - 1) / (uint32_t)kRedGroup;
    const uint32_t gfirst = group * (uint32_t)kRedGroup;
    const uint32_t gsize = min((uint32_t)kRedGroup, nblocks - gfirst);
    double *gpart = partial + (size_t)nblocks * width;  // group partials, after the blocks'
    __shared__ unsigned ticket;

    // sum `count` rows of src (row stride width) starting at row `first` into red[0..width)
    auto sum_rows = [&](const double *src, uint32_t first, uint32_t count) {
        for (int k = tid; k < T * width; k += nt) {
            const int s = k / width, q = k - s * width;
            double a0 = 0.0, a1 = 0.0;
            uint32_t b = (uint32_t)s;
            for (; b + (uint32_t)T < count; b += 2u * T) {
                a0 += src[(size_t)(first + b) * width + q];
                a1 += src[(size_t)(first + b + T) * width + q];
            }
            for (; b < count; b += T) a0 += src[(size_t)(first + b) * width + q];
            red[k] = a0 + a1;
        }
        __syncthreads();
        for (int w = T >> 1; w > 0; w >>= 1) {
            for (int k = tid; k < w * width; k += nt) red[k] += red[k + w * width];
            __syncthreads();
        }
    };

    __threadfence();
    __syncthreads();
    if (tid == 0)
        ticket = __hip_atomic_fetch_add(counter + 1 + group, 1u, __ATOMIC_ACQ_REL,
                                        __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (ticket != gsize - 1) return;
    __threadfence();
    // last block of the group: the group's partials in block order
    sum_rows(partial, gfirst, gsize);
    if (tid == 0) __hip_atomic_store(counter + 1 + group, 0u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    if (ngroups == 1) {
        for (int k = tid; k < width; k += nt) result[k] = red[k];
        return;
    }
    for (int k = tid; k < width; k += nt) gpart[(size_t)group * width + k] = red[k];
    __threadfence();
    __syncthreads();
    if (tid == 0)
        ticket = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (ticket != ngroups - 1) return;
    __threadfence();
    // last group: the group sums in group order
    sum_rows(gpart, 0, ngroups);
    for (int k = tid; k < width; k += nt) result[k] = red[k];
    if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace cola
