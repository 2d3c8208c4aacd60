// Site-structured vector kernels for the CG solvers.  One lane owns one
// (site, rhs) pair and all 12 of its spin-colour components, so FP16 blocks
// can rescale per site and every per-rhs scalar (alpha, beta, scale) is one
// register.  Consecutive lanes take consecutive (site, rhs) pairs, which in
// the rhs-innermost packed layout are consecutive addresses for every
// component.  Reductions are per rhs, in FP64, deterministic.
#include "cola.h"
#include "device.h"
#include "launch.h"

namespace cola {

namespace {

size_t block_bytes(SpinorFmt f, int S, int R) {
    const size_t SR = (size_t)S * R;
    switch (f) {
        case SpinorFmt::F64: return 12 * SR * 16;
        case SpinorFmt::F32: return 12 * SR * 8;
        default: return 12 * SR * 4 + SR * 4;
    }
}

struct Loc {
    uint32_t blk, i, r;
};

// The parity block of a lane is blockIdx.y, so every view is wavefront-uniform.
template <SpinorFmt F>
__device__ __forceinline__ SpinorBlock<F, true> view(const void *base, size_t bb, const Loc &l,
                                                     int S, int R) {
    return SpinorBlock<F, true>((const char *)base + l.blk * bb, S, R);
}

// Generic grid-stride driver over one parity block per grid row (blockIdx.y):
// f(loc) returns this lane's contribution to the per-rhs reduction (ignored when
// red.result is null).
template <class Fn>
__global__ void __launch_bounds__(256) site_kernel(Fn f, const BlasShape sh, const Reduce red) {
    extern __shared__ double lds[];
    const uint32_t SR = (uint32_t)sh.S * sh.R;
    double acc[1] = {0.0};
    Loc l;
    l.blk = blockIdx.y;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < SR; e += gridDim.x * blockDim.x) {
        l.i = e / (uint32_t)sh.R;
        l.r = e - l.i * (uint32_t)sh.R;
        acc[0] += f(l);
    }
    if (red.result) {
        const int slot = threadIdx.x / sh.R;
        const int q = threadIdx.x - slot * sh.R;
        block_sum_to_partial<1>(lds, sh.T, sh.R, slot, q, 1, acc, red.partial,
                                blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    }
}

hipError_t launch_reduce(const double *partial, int nblocks, int width, double *result,
                         hipStream_t st);

template <class Fn>
hipError_t run(const Fn &f, const BlasShape &sh, const Reduce *red, hipStream_t st) {
    Reduce r = red ? *red : Reduce{nullptr, nullptr, nullptr};
    const size_t shm = r.result ? (size_t)sh.T * sh.R * sizeof(double) : 0;
    hipLaunchKernelGGL(site_kernel<Fn>, dim3(sh.grid, sh.nblk), dim3(sh.T * sh.R), shm, st, f,
                       sh, r);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && r.result)
        e = launch_reduce(r.partial, sh.grid * sh.nblk, sh.R, r.result, st);
    return e;
}

template <SpinorFmt FX, SpinorFmt FP, SpinorFmt FR, SpinorFmt FA>
struct XrFn {
    void *x;
    const void *p;
    void *r;
    const void *ap;
    size_t bx, bp, br, ba;
    const double *rho, *pi, *pi2;
    const int *active;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        using TX = typename SpinorT<FX>::real;
        using TR = typename SpinorT<FR>::real;
        const double den = pi[l.r] + (pi2 ? pi2[l.r] : 0.0);
        const double al = active[l.r] && den != 0.0 ? rho[l.r] / den : 0.0;
        const auto X = view<FX>(x, bx, l, S, R);
        const auto P = view<FP>(p, bp, l, S, R);
        const auto Rv = view<FR>(r, br, l, S, R);
        const auto A = view<FA>(ap, ba, l, S, R);
        cpx<TX> xv[12];
        cpx<typename SpinorT<FP>::real> pv[12];
        cpx<TR> rv[12];
        cpx<typename SpinorT<FA>::real> av[12];
        X.load(l.i, l.r, xv);
        P.load(l.i, l.r, pv);
        Rv.load(l.i, l.r, rv);
        A.load(l.i, l.r, av);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            xv[c].x += (TX)al * (TX)pv[c].x;
            xv[c].y += (TX)al * (TX)pv[c].y;
            rv[c].x -= (TR)al * (TR)av[c].x;
            rv[c].y -= (TR)al * (TR)av[c].y;
        }
        X.store(l.i, l.r, xv);
        Rv.store(l.i, l.r, rv);
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) s += (double)norm2(rv[c]);
        return s;
    }
};

template <SpinorFmt FR, SpinorFmt FP>
struct PFn {
    const void *r;
    void *p;
    size_t br, bp;
    const double *rho_new, *rho;
    const int *active;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        using TP = typename SpinorT<FP>::real;
        const double be = active[l.r] && rho[l.r] != 0.0 ? rho_new[l.r] / rho[l.r] : 0.0;
        const auto Rv = view<FR>(r, br, l, S, R);
        const auto P = view<FP>(p, bp, l, S, R);
        cpx<typename SpinorT<FR>::real> rv[12];
        cpx<TP> pv[12];
        Rv.load(l.i, l.r, rv);
        P.load(l.i, l.r, pv);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            pv[c].x = (TP)rv[c].x + (TP)be * pv[c].x;
            pv[c].y = (TP)rv[c].y + (TP)be * pv[c].y;
        }
        P.store(l.i, l.r, pv);
        return 0.0;
    }
};

template <SpinorFmt F>
struct NormFn {
    const void *v;
    size_t bv;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        cpx<typename SpinorT<F>::real> a[12];
        view<F>(v, bv, l, S, R).load(l.i, l.r, a);
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) s += (double)norm2(a[c]);
        return s;
    }
};

template <SpinorFmt FD, SpinorFmt FS>
struct ConvFn {
    void *d;
    const void *s;
    size_t bd, bs;
    const double *scale;
    int inv;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        using TD = typename SpinorT<FD>::real;
        cpx<typename SpinorT<FS>::real> a[12];
        view<FS>(s, bs, l, S, R).load(l.i, l.r, a);
        double f = 1.0;
        if (scale) f = inv ? (scale[l.r] != 0.0 ? 1.0 / scale[l.r] : 0.0) : scale[l.r];
        cpx<TD> o[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = {(TD)(f * (double)a[c].x), (TD)(f * (double)a[c].y)};
        view<FD>(d, bd, l, S, R).store(l.i, l.r, o);
        double n = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) n += (double)norm2(o[c]);
        return n;
    }
};

template <SpinorFmt FS>
struct AccumFn {
    void *d;
    void *s;
    size_t bd, bs;
    const double *scale;
    int zero;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        using TS = typename SpinorT<FS>::real;
        const auto Sv = view<FS>(s, bs, l, S, R);
        const auto D = view<SpinorFmt::F64>(d, bd, l, S, R);
        cpx<TS> a[12];
        cpx<double> o[12];
        Sv.load(l.i, l.r, a);
        D.load(l.i, l.r, o);
        const double f = scale ? scale[l.r] : 1.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            o[c].x = fma(f, (double)a[c].x, o[c].x);
            o[c].y = fma(f, (double)a[c].y, o[c].y);
        }
        D.store(l.i, l.r, o);
        if (zero) {
#pragma unroll
            for (int c = 0; c < 12; ++c) a[c] = {(TS)0, (TS)0};
            Sv.store(l.i, l.r, a);
        }
        return 0.0;
    }
};

struct ResidualFn {
    void *r;
    const void *b, *ax;
    size_t bb;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        cpx<double> bv[12], av[12];
        view<SpinorFmt::F64>(b, bb, l, S, R).load(l.i, l.r, bv);
        view<SpinorFmt::F64>(ax, bb, l, S, R).load(l.i, l.r, av);
        double n = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            bv[c] = bv[c] - av[c];
            n += norm2(bv[c]);
        }
        view<SpinorFmt::F64>(r, bb, l, S, R).store(l.i, l.r, bv);
        return n;
    }
};

template <SpinorFmt F, typename CR>
struct CloverFn {
    void *out;
    const void *in;
    const void *clov;
    size_t bb;
    int parity;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        using T = typename SpinorT<F>::real;
        cpx<T> a[12], o[12];
        view<F>(in, bb, l, S, R).load(l.i, l.r, a);
        clover_apply<CR, T>(clov, S, parity, l.i, a, o);
        view<F>(out, bb, l, S, R).store(l.i, l.r, o);
        return 0.0;
    }
};

}  // namespace

namespace {

// result[q] = sum over b < nblocks of partial[q * nblocks + b], in a fixed order: one
// block of 1024 threads per column; thread t adds blocks t + 1024 k in eight independent
// chains (the loads overlap), then an LDS tree adds the threads.
__global__ void __launch_bounds__(1024) reduce_partials_kernel(const double *partial,
                                                               int nblocks, double *result) {
    __shared__ double red[1024];
    const int q = blockIdx.x;
    const int t = threadIdx.x;
    const double *col = partial + (size_t)q * nblocks;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = t;
    for (; b + 7 * 1024 < nblocks; b += 8 * 1024) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += col[b + k * 1024];
    }
    for (; b < nblocks; b += 1024) a[0] += col[b];
    red[t] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) result[q] = red[0];
}

}  // namespace

hipError_t launch_reduce_partials(const double *partial, int nblocks, int width, double *result,
                                  hipStream_t st) {
    return launch_reduce(partial, nblocks, width, result, st);
}

namespace {

hipError_t launch_reduce(const double *partial, int nblocks, int width, double *result,
                         hipStream_t st) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(width), dim3(1024), 0, st, partial, nblocks,
                       result);
    return hipGetLastError();
}

}  // namespace

BlasShape blas_shape(const Geom &g, int nrhs, int nblk) {
    BlasShape b;
    b.S = g.S;
    b.R = nrhs;
    b.nblk = nblk;
    int T = 1;
    while (T * 2 * nrhs <= 256) T *= 2;
    b.T = T;
    const size_t work = (size_t)g.S * nrhs;  // per parity block (grid row)
    size_t grid = (work + (size_t)T * nrhs - 1) / ((size_t)T * nrhs);
    // at most kRedMaxBlocks blocks over all rows (the partial-sum array); grid-stride beyond
    const size_t cap = (size_t)kRedMaxBlocks / (size_t)(nblk < 1 ? 1 : nblk);
    if (grid > cap) grid = cap;
    b.grid = (int)(grid < 1 ? 1 : grid);
    return b;
}

#define DISPATCH_FMT(f, FT, ...)                                     \
    switch (f) {                                                     \
        case SpinorFmt::F64: { constexpr SpinorFmt FT = SpinorFmt::F64; __VA_ARGS__; } break; \
        case SpinorFmt::F32: { constexpr SpinorFmt FT = SpinorFmt::F32; __VA_ARGS__; } break; \
        case SpinorFmt::F16: { constexpr SpinorFmt FT = SpinorFmt::F16; __VA_ARGS__; } break; \
    }

namespace {
struct MsFn {
    void *x, *p;
    const void *r;
    size_t bx, br;
    const MsCoef *kp;
    int S, R;
    __device__ double operator()(const Loc &l) const {
        const MsCoef &k = *kp;
        if (!k.active[l.r]) return 0.0;
        const auto X = view<SpinorFmt::F64>(x, bx, l, S, R);
        const auto P = view<SpinorFmt::F64>(p, bx, l, S, R);
        const auto Rv = view<SpinorFmt::F64>(r, br, l, S, 1);
        cpx<double> xv[12], pv[12], rv[12];
        X.load(l.i, l.r, xv);
        P.load(l.i, l.r, pv);
        Rv.load(l.i, 0, rv);
        const double a = k.alpha[l.r], z = k.zeta[l.r], b = k.beta[l.r];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            xv[c] = {fma(a, pv[c].x, xv[c].x), fma(a, pv[c].y, xv[c].y)};
            pv[c] = {fma(z, rv[c].x, b * pv[c].x), fma(z, rv[c].y, b * pv[c].y)};
        }
        X.store(l.i, l.r, xv);
        P.store(l.i, l.r, pv);
        return 0.0;
    }
};

struct MsResFn {
    const void *b, *ax, *x;
    size_t bb, bx;
    double sigma[kRedMaxWidth];
    int S, R;
    __device__ double operator()(const Loc &l) const {
        const auto B = view<SpinorFmt::F64>(b, bb, l, S, 1);
        const auto AX = view<SpinorFmt::F64>(ax, bx, l, S, R);
        const auto X = view<SpinorFmt::F64>(x, bx, l, S, R);
        cpx<double> bv[12], av[12], xv[12];
        B.load(l.i, 0, bv);
        AX.load(l.i, l.r, av);
        X.load(l.i, l.r, xv);
        const double sg = sigma[l.r];
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double re = bv[c].x - av[c].x - sg * xv[c].x;
            const double im = bv[c].y - av[c].y - sg * xv[c].y;
            s += re * re + im * im;
        }
        return s;
    }
};

__global__ void scalar_add_kernel(double *a, const double *b, int n) {
    const int i = (int)threadIdx.x;
    if (i < n) a[i] += b[i];
}
__global__ void scalar_copy_kernel(double *a, const double *b, int n) {
    const int i = (int)threadIdx.x;
    if (i < n) a[i] = b[i];
}
}  // namespace

hipError_t launch_ms_update(const BlasShape &sh, void *x, void *p, const void *r,
                            const MsCoef *k, hipStream_t st) {
    MsFn fn{x, p, r, block_bytes(SpinorFmt::F64, sh.S, sh.R), block_bytes(SpinorFmt::F64, sh.S, 1),
            k, sh.S, sh.R};
    return run(fn, sh, nullptr, st);
}

namespace {

struct MsShifts {
    double sigma[kRedMaxWidth];
};

__global__ void ms_init_kernel(MsState *st, MsShifts sh, int nshift, double tol2,
                               const double *bnorm) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double b2 = *bnorm;
    st->nshift = nshift;
    st->alpha_old = 1.0;
    st->beta_old = 0.0;
    st->rho = b2;
    st->thr = tol2 * b2;
    st->status = COLA_OK;
    st->iterations = 0;
    int all = 1;
    for (int q = 0; q < kRedMaxWidth; ++q) {
        const bool live = q < nshift;
        st->sigma[q] = live ? sh.sigma[q] : 0.0;
        st->zeta[q] = 1.0;
        st->zold[q] = 1.0;
        st->done[q] = live ? (b2 == 0.0 ? 1 : 0) : 1;
        all &= st->done[q];
        // the first update: p_q = b (alpha 0, zeta 1, beta 0)
        st->coef.alpha[q] = 0.0;
        st->coef.zeta[q] = 1.0;
        st->coef.beta[q] = 0.0;
        st->coef.active[q] = live ? 1 : 0;
    }
    st->finished = all;
}

// One iteration of the shifted recursion (the host loop it replaces ran the same
// arithmetic in the same order):
//   zeta_q' = zeta_q zeta_q^old alpha^old /
//             (alpha beta^old (zeta_q^old - zeta_q) + zeta_q^old alpha^old (1 + sigma_q alpha))
//   alpha_q = alpha zeta_q'/zeta_q, beta_q = beta (zeta_q'/zeta_q)^2; shifts done
//   (zeta_q^2 |r|^2 <= tol^2 |b|^2) stay frozen.
__global__ void ms_advance_kernel(MsState *st, const double *rho_new_p, const double *pi_p,
                                  const double *pi2_p) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    MsCoef &k = st->coef;
    if (st->finished || st->status != COLA_OK) {
        for (int q = 0; q < kRedMaxWidth; ++q) k.active[q] = 0;
        return;
    }
    const double rho = st->rho, rho_new = *rho_new_p;
    const double pi = *pi_p + (pi2_p ? *pi2_p : 0.0);
    const double alpha = rho / pi, beta = rho_new / rho;
    if (!isfinite(alpha) || !isfinite(beta) || !(pi > 0.0)) {
        st->status = COLA_BREAKDOWN;
        for (int q = 0; q < kRedMaxWidth; ++q) k.active[q] = 0;
        return;
    }
    bool bad = false;
    for (int q = 0; q < st->nshift; ++q) {
        k.active[q] = !st->done[q];
        const double z = st->zeta[q], zo = st->zold[q];
        double zn = z;
        if (!st->done[q]) {  // done shifts are frozen (their zeta may underflow)
            zn = z * zo * st->alpha_old /
                 (alpha * st->beta_old * (zo - z) + zo * st->alpha_old * (1.0 + st->sigma[q] * alpha));
            k.alpha[q] = alpha * zn / z;
            k.zeta[q] = zn;
            k.beta[q] = beta * (zn / z) * (zn / z);
            bad |= !isfinite(zn);
        }
        st->zold[q] = z;
        st->zeta[q] = zn;
    }
    if (bad) {
        st->status = COLA_BREAKDOWN;
        for (int q = 0; q < kRedMaxWidth; ++q) k.active[q] = 0;
        return;
    }
    st->alpha_old = alpha;
    st->beta_old = beta;
    st->rho = rho_new;
    st->iterations += 1;
    int all = 1;
    for (int q = 0; q < st->nshift; ++q) {
        if (st->zeta[q] * st->zeta[q] * rho_new <= st->thr) st->done[q] = 1;
        all &= st->done[q];
    }
    st->finished = all;
}

}  // namespace

hipError_t launch_ms_init(MsState *state, const double *sigma, int nshift, double tol2,
                          const double *bnorm, hipStream_t st) {
    if (nshift < 1 || nshift > kRedMaxWidth) return hipErrorInvalidValue;
    MsShifts sh{};
    for (int q = 0; q < nshift; ++q) sh.sigma[q] = sigma[q];
    hipLaunchKernelGGL(ms_init_kernel, dim3(1), dim3(64), 0, st, state, sh, nshift, tol2, bnorm);
    return hipGetLastError();
}

hipError_t launch_ms_advance(MsState *state, const double *rho_new, const double *pi,
                             const double *pi2, hipStream_t st) {
    hipLaunchKernelGGL(ms_advance_kernel, dim3(1), dim3(64), 0, st, state, rho_new, pi, pi2);
    return hipGetLastError();
}

hipError_t launch_ms_residual(const BlasShape &sh, const void *b, const void *ax, const void *x,
                              const double *sigma, const Reduce &red, hipStream_t st) {
    MsResFn fn{b, ax, x, block_bytes(SpinorFmt::F64, sh.S, 1),
               block_bytes(SpinorFmt::F64, sh.S, sh.R), {}, sh.S, sh.R};
    for (int q = 0; q < sh.R && q < kRedMaxWidth; ++q) fn.sigma[q] = sigma[q];
    return run(fn, sh, &red, st);
}

hipError_t launch_scalar_add(double *a, const double *b, int n, hipStream_t st) {
    hipLaunchKernelGGL(scalar_add_kernel, dim3(1), dim3(64), 0, st, a, b, n);
    return hipGetLastError();
}

hipError_t launch_scalar_copy(double *a, const double *b, int n, hipStream_t st) {
    if (n < 0 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scalar_copy_kernel, dim3(1), dim3(64), 0, st, a, b, n);
    return hipGetLastError();
}

hipError_t launch_cg_xr(const BlasShape &b, SpinorFmt fx, SpinorFmt fp, SpinorFmt fr,
                        SpinorFmt fap, void *x, const void *p, void *r, const void *ap,
                        const double *rho, const double *pi, const double *pi2,
                        const int *active, const Reduce &red, hipStream_t st) {
    // supported combinations: all equal, or (x FP32, p FP16, r FP32, Ap FP16)
    if (fx == fp && fp == fr && fr == fap) {
        DISPATCH_FMT(fx, F,
                     XrFn<F, F, F, F> fn{x, p, r, ap, block_bytes(F, b.S, b.R), block_bytes(F, b.S, b.R),
                                         block_bytes(F, b.S, b.R), block_bytes(F, b.S, b.R),
                                         rho, pi, pi2, active, b.S, b.R};
                     return run(fn, b, &red, st));
    }
    if (fx == SpinorFmt::F32 && fp == SpinorFmt::F16 && fr == SpinorFmt::F32 &&
        fap == SpinorFmt::F16) {
        XrFn<SpinorFmt::F32, SpinorFmt::F16, SpinorFmt::F32, SpinorFmt::F16> fn{
            x, p, r, ap,
            block_bytes(SpinorFmt::F32, b.S, b.R), block_bytes(SpinorFmt::F16, b.S, b.R),
            block_bytes(SpinorFmt::F32, b.S, b.R), block_bytes(SpinorFmt::F16, b.S, b.R),
            rho, pi, pi2, active, b.S, b.R};
        return run(fn, b, &red, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_cg_p(const BlasShape &b, SpinorFmt fr, SpinorFmt fp, const void *r, void *p,
                       const double *rho_new, const double *rho, const int *active,
                       hipStream_t st) {
    if (fr == fp) {
        DISPATCH_FMT(fr, F,
                     PFn<F, F> fn{r, p, block_bytes(F, b.S, b.R), block_bytes(F, b.S, b.R),
                                  rho_new, rho, active, b.S, b.R};
                     return run(fn, b, nullptr, st));
    }
    if (fr == SpinorFmt::F32 && fp == SpinorFmt::F16) {
        PFn<SpinorFmt::F32, SpinorFmt::F16> fn{r, p, block_bytes(fr, b.S, b.R),
                                               block_bytes(fp, b.S, b.R), rho_new, rho, active,
                                               b.S, b.R};
        return run(fn, b, nullptr, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_norm2(const BlasShape &b, SpinorFmt f, const void *v, const Reduce &red,
                        hipStream_t st) {
    DISPATCH_FMT(f, F, NormFn<F> fn{v, block_bytes(F, b.S, b.R), b.S, b.R};
                 return run(fn, b, &red, st));
    return hipErrorInvalidValue;
}

hipError_t launch_convert(const BlasShape &b, SpinorFmt fd, SpinorFmt fs, void *dst,
                          const void *src, const double *s, int inv_scale, const Reduce *red,
                          hipStream_t st) {
    DISPATCH_FMT(fd, FD, DISPATCH_FMT(fs, FS,
                 ConvFn<FD, FS> fn{dst, src, block_bytes(FD, b.S, b.R), block_bytes(FS, b.S, b.R),
                                   s, inv_scale, b.S, b.R};
                 return run(fn, b, red, st)));
    return hipErrorInvalidValue;
}

hipError_t launch_accum(const BlasShape &b, SpinorFmt fs, void *dst, void *src, const double *s,
                        int zero_src, hipStream_t st) {
    DISPATCH_FMT(fs, FS,
                 AccumFn<FS> fn{dst, src, block_bytes(SpinorFmt::F64, b.S, b.R),
                                block_bytes(FS, b.S, b.R), s, zero_src, b.S, b.R};
                 return run(fn, b, nullptr, st));
    return hipErrorInvalidValue;
}

hipError_t launch_residual(const BlasShape &b, void *r, const void *bb, const void *ax,
                           const Reduce &red, hipStream_t st) {
    ResidualFn fn{r, bb, ax, block_bytes(SpinorFmt::F64, b.S, b.R), b.S, b.R};
    return run(fn, b, &red, st);
}

hipError_t launch_clover_site(const BlasShape &b, SpinorFmt f, int clov_double, void *out,
                              const void *in, const void *clov, int parity, hipStream_t st) {
    if (clov_double) {
        DISPATCH_FMT(f, F, CloverFn<F, double> fn{out, in, clov, block_bytes(F, b.S, b.R),
                                                  parity, b.S, b.R};
                     return run(fn, b, nullptr, st));
    } else {
        DISPATCH_FMT(f, F, CloverFn<F, float> fn{out, in, clov, block_bytes(F, b.S, b.R),
                                                 parity, b.S, b.R};
                     return run(fn, b, nullptr, st));
    }
    return hipErrorInvalidValue;
}

}  // namespace cola
