// Half-lattice Wilson hopping term for gfx950 (kernel template; each
// precision is instantiated in its own translation unit).
//
// One lane owns one output site of parity p and RPT of its right-hand sides;
// consecutive lanes take the right-hand-side groups of one site, then the
// next site, so a site's link is fetched by neighbouring lanes of one
// wavefront (one memory transaction) and reused from registers across the
// lane's RPT right-hand sides.  Per direction: load the link (rows 0-1 for the
// compressed formats, row 2 rebuilt in registers), load the neighbour spinor,
// project it to two spin components with (1 -+ g_mu), multiply both colour
// vectors by U or U^H, apply the boundary phase and expand back into the four
// spin components.  Real boundary phases (theta = 0 or pi) fold into the
// accumulation sign; complex ones are a complex multiply.  The epilogue is a
// template parameter:
//   EPI_NONE       out = D in
//   EPI_XPAY       out = x + a D in
//   EPI_CLOV       out = C (D in)
//   EPI_CLOV_XPAY  out = C x + a D in
//   EPI_XPAY_CLOV  out = C (x + a D in)
//   EPI_XPAY_CG, EPI_CLOV_XPAY_CG: the CG update of x and r with o = x + a D in
//                  (or C x + a D in) in place of storing o
// and |out|^2 per rhs can be accumulated: per-block partials, summed in block
// order by a reduce_partials launch that follows.
//
// Time walk (one rhs per lane, links staged in LDS): a lane keeps the same
// (xh, y, z) and walks the timeslices of its chunk.  The input sites with the lane's own
// checkerboard index at t - 1, t and t + 1 are its two time neighbours and one of its
// two x neighbours, and each of them is needed again one or two steps later, so they
// stay in registers: a step loads the t + 1 site and the other x, y and z neighbours
// (six spinors instead of eight), and the reuse that otherwise depends on a site staying
// in L2 for a whole step of the walk is certain.  These kernels (FP32 and FP16, used when
// a lane walks more than one timeslice) run at three waves per SIMD to hold the extra
// spinors.  Every kernel adds the eight directions in the same
// order (t backward first), so all launch shapes give bitwise the same result.
//
// FL (the fat-link irrelevant clover operator): the hop of direction mu is
// (F - g_mu U) psi(x+mu) forward and (F^H + g_mu U^H) psi(x-mu) backward, with U the
// thin links (a.gauge) and F the smeared links (a.gauge_fat).  Writing
// 1 = (1 + g)/2 + (1 - g)/2, the term of the projector (1 + s g_mu) (s = +-1) carries
// the link F + s sg U, where (1 + sg g_mu) is the Wilson projector of that direction
// (the same sign conventions, dagger included), so each direction costs two spin
// projections and four SU(3) products of the combined links F +- U.
#pragma once

#include <type_traits>

#include "device.h"
#include "launch.h"

namespace cola {

// The neighbour spinor of one direction as loaded: raw halves and site scales for FP16,
// compute-precision components otherwise; n is the neighbour's checkerboard index.
template <SpinorFmt SF, int RPT>
struct Fetched {
    using T = typename SpinorT<SF>::real;
    using E = typename std::conditional<SF == SpinorFmt::F16, h2, cpx<T>>::type;
    E s[RPT][12];
    float scl[RPT];
    uint32_t n;
};

// Issue the loads of direction (MU, DIR)'s neighbour spinor.  The kernel fetches one
// direction ahead of the one it computes, so a wavefront always has a direction's
// loads in flight while it does arithmetic (the register fences between directions are
// scheduling barriers: without this the loads of a direction would only start after
// the previous direction finished).
template <int MU, int DIR, SpinorFmt SF, int RPT>
__device__ __forceinline__ void hop_fetch(const HopArgs &a, const SpinorBlock<SF, true> &in,
                                          uint32_t i, const int x[4], uint32_t j,
                                          Fetched<SF, RPT> &f) {
    const Geom &g = a.g;
    f.n = DIR == 0 ? nb_fwd(g, i, x, MU) : nb_bwd(g, i, x, MU);
    if constexpr (SF == SpinorFmt::F16) {
        in.template load_raw_h2_group<RPT>(f.n, j * RPT, f.s, f.scl);
    } else {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            typename SpinorT<SF>::real one;  // the site scale, 1 for FP32 and FP64 blocks
            in.load_unscaled(f.n, j * RPT + r, f.s[r], &one);
        }
    }
}

// the spinor of site n (rhs j) into f, one rhs per lane (FP16: raw halves and scale)
template <SpinorFmt SF>
__device__ __forceinline__ void fetch_site(const SpinorBlock<SF, true> &in, uint32_t n, uint32_t j,
                                           Fetched<SF, 1> &f) {
    f.n = n;
    if constexpr (SF == SpinorFmt::F16) {
        in.template load_raw_h2_group<1>(n, j, f.s, f.scl);
    } else {
        typename SpinorT<SF>::real one;
        in.load_unscaled(n, j, f.s[0], &one);
    }
}

// The order in which the eight directions d = 2 mu + dir are added: t backward first,
// then x, y, z and t forward (the time walk has the t backward neighbour in registers
// at the start of a step).
constexpr int hop_order(int k) { return k == 0 ? 7 : k - 1; }

// One of the eight hopping directions (MU, DIR) added into the accumulators of the
// lane's RPT right-hand sides at checkerboard site i (coordinates x), from the fetched
// neighbour spinor.  A template, so the eight directions are unrolled by construction
// and every spin-projection branch resolves at compile time.
template <int MU, int DIR, SpinorFmt SF, LinkFmt LF, int RPT, bool RPH, bool SHL, bool FL>
__device__ __forceinline__ void hop_dir(const HopArgs &a, int p, uint32_t i, const int x[4],
                                        typename SpinorT<SF>::real sg_f,
                                        cpx<typename SpinorT<SF>::real> acc[RPT][12],
                                        const uint32_t *staged, const Fetched<SF, RPT> &f) {
    using T = typename SpinorT<SF>::real;
    using C = cpx<T>;
    const Geom &g = a.g;
    constexpr int mu = MU, dir = DIR;
    const T sg_b = -sg_f;
    // dir 0: (1 + sg_f g_mu) e+ U_mu(x) psi(x+mu)
    // dir 1: (1 + sg_b g_mu) e- U_mu(x-mu)^H psi(x-mu)
    const uint32_t n = f.n;
    const T sg = dir == 0 ? sg_f : sg_b;
    const bool bnd = dir == 0 ? x[mu] == g.L[mu] - 1 : x[mu] == 0;
    T eta = (T)1;
    C ph = {(T)1, (T)0};
    if constexpr (RPH) {
        eta = bnd ? (T)a.phase[mu].x : (T)1;
    } else {
        const T im = dir == 0 ? (T)a.phase[mu].y : -(T)a.phase[mu].y;
        ph = bnd ? C{(T)a.phase[mu].x, im} : C{(T)1, (T)0};
    }
    if constexpr (FL) {
        static_assert(SF != SpinorFmt::F16 && !SHL, "FLIC hops: FP64 / FP32, per-lane links");
        C u[3][3], fl[3][3];
        const int lpar = dir == 0 ? p : 1 - p;
        const uint32_t li = dir == 0 ? i : n;
        load_link<LF, T>(a.gauge, g.S, lpar, mu, li, u);
        load_link<LF, T>(a.gauge_fat, g.S, lpar, mu, li, fl);
        // in place: fl = F + U (with the projector 1 + sg g_mu), u = F - U (1 - sg g_mu)
#pragma unroll
        for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
            for (int c0 = 0; c0 < 3; ++c0) {
                const C f0 = fl[r0][c0];
                fl[r0][c0] = f0 + u[r0][c0];
                u[r0][c0] = f0 - u[r0][c0];
            }
        const T half = (T)0.5 * eta;
        auto term = [&](const C (&L)[3][3], T sp) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                C h[6], w[6];
                project(mu, sp, f.s[r], h);
                if constexpr (dir == 0) {
                    su3_mul(L, h, w);
                    su3_mul(L, h + 3, w + 3);
                } else {
                    su3_dag_mul(L, h, w);
                    su3_dag_mul(L, h + 3, w + 3);
                }
                if constexpr (!RPH) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) w[k] = cmul(ph, w[k]);
                }
                expand_add(mu, sp, w, acc[r], half);
            }
        };
        term(fl, sg);
        term(u, -sg);
    } else if constexpr (SF == SpinorFmt::F16) {
        // packed-half projection and dot2 products: FP16 x FP16 products are exact
        // and summed in FP32; the per-site scale rides on eta.  The link operands are
        // prepared once for the lane's RPT right-hand sides, which are adjacent in
        // memory: one wide load per component.
        LinkH2 L;
        if constexpr (SHL)
            read_staged(staged + (2 * MU + DIR) * kStageWords, L);
        else
            load_link_h2<dir == 1>(a.gauge, g.S, dir == 0 ? p : 1 - p, mu, dir == 0 ? i : n, L);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            h2 hh[6];
            C w[6];
            project_h2(mu, (_Float16)sg, f.s[r], hh);
            mul_h2(L, hh, w);
            mul_h2(L, hh + 3, w + 3);
            if constexpr (!RPH) {
#pragma unroll
                for (int k = 0; k < 6; ++k) w[k] = cmul(ph, w[k]);
            }
            expand_add(mu, sg, w, acc[r], eta * f.scl[r]);
        }
    } else {
        C u[3][3];
        if constexpr (SHL && LF == LinkFmt::F32_12)
            read_staged(staged + (2 * MU + DIR) * kStageWords, u);
        else if (a.groups == 1)  // one lane per site: each link is read by one lane only
            load_link<LF, T, true, kCpolNT>(a.gauge, g.S, dir == 0 ? p : 1 - p, mu,
                                            dir == 0 ? i : n, u);
        else
            load_link<LF, T>(a.gauge, g.S, dir == 0 ? p : 1 - p, mu, dir == 0 ? i : n, u);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            C h[6], w[6];
            project(mu, sg, f.s[r], h);
            if constexpr (dir == 0) {
                su3_mul(u, h, w);
                su3_mul(u, h + 3, w + 3);
            } else {
                su3_dag_mul(u, h, w);
                su3_dag_mul(u, h + 3, w + 3);
            }
            if constexpr (!RPH) {
#pragma unroll
                for (int k = 0; k < 6; ++k) w[k] = cmul(ph, w[k]);
            }
            expand_add(mu, sg, w, acc[r], eta);
        }
    }
    // Register fence: the accumulators are final for this direction here, so the
    // compiler cannot sink a direction's arithmetic to the end of the kernel (which
    // kept every loaded spinor and link live at once).
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(acc[r][c].x), "+v"(acc[r][c].y));
}

// The kernels that can walk time with neighbours in registers: FP32 and FP16 spinors,
// one rhs per lane, staged links, not the CG-update epilogues (whose x, p and r would
// not fit beside the carried spinors).  They walk (a second instantiation, WK) when a
// lane has more than one timeslice to walk.
template <SpinorFmt SF, int RPT, int EPI, bool SHL, bool FL>
constexpr bool hop_walks() {
    return (SF == SpinorFmt::F32 || SF == SpinorFmt::F16) && RPT == 1 && SHL && !FL &&
           EPI != EPI_XPAY_CG && EPI != EPI_CLOV_XPAY_CG;
}

template <SpinorFmt SF, LinkFmt LF, typename CR, int RPT, int EPI, bool RPH, bool SHL,
          bool FL = false, bool WK = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WK ? 3 : 1)))
    hop_kernel(const HopArgs a) {
    using T = typename SpinorT<SF>::real;
    using C = cpx<T>;
    constexpr bool WALK = WK;
    static_assert(!WK || hop_walks<SF, RPT, EPI, SHL, FL>(), "no time walk for this kernel");
    extern __shared__ double red[];
    // SHL: the site's eight links staged in LDS by its first eight lanes, and with a clover
    // epilogue (FP32 blocks) the site's clover block by all its lanes
    constexpr bool CLV = EPI == EPI_CLOV || EPI == EPI_CLOV_XPAY || EPI == EPI_XPAY_CLOV ||
                         EPI == EPI_CLOV_XPAY_CG;
    constexpr bool SCL = SHL && CLV && std::is_same<CR, float>::value;
    __shared__ __attribute__((aligned(16))) uint32_t stage[SHL ? kStageSites * kStageSite : 4];
    __shared__ __attribute__((aligned(16))) float cstage[SCL ? kStageSites * kClovStage : 4];
    const Geom &g = a.g;
    const int p = a.parity;
    const SpinorBlock<SF, true> in(a.in, g.S, a.nrhs);
    const SpinorBlock<SF, true> out(a.out, g.S, a.nrhs);
    const SpinorBlock<SF, true> xin(a.x ? a.x : a.out, g.S, a.nrhs);
    const SpinorBlock<SF, true> cgx(a.cg_x ? a.cg_x : a.out, g.S, a.nrhs);
    const SpinorBlock<SF, true> cgr(a.cg_r ? a.cg_r : a.out, g.S, a.nrhs);
    const SpinorBlock<SF, true> cgp(a.cg_p ? a.cg_p : a.out, g.S, a.nrhs);
    const T sg_f = a.dagger ? (T)1 : (T)-1;
    double nrm[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) nrm[r] = 0.0;

    // Work is cut into blockDim-lane chunks; each XCD (blocks are dispatched to the 8
    // XCDs round-robin) takes one contiguous range of chunks, in proportion to its
    // blocks, and its blocks stride over that range only: neighbouring sites stay in
    // that XCD's L2 whether the grid covers the work once or loops over it.
    uint32_t c0, c1, cstep, cfirst;
    xcd_range(blockIdx.x, gridDim.x, (a.total + blockDim.x - 1) / blockDim.x, &c0, &c1, &cstep);
    cfirst = c0;
    const uint32_t ncol = (uint32_t)g.s3;  // checkerboard sites of one timeslice
    // Lane w owns rhs group j of spatial column c in time chunk k and walks the chunk's
    // timeslices: the spinors its t-neighbours need were fetched one step earlier.  The
    // trip count is the same for every lane of a block (lanes past the end idle), so the
    // staging barriers are reached by all.
    for (uint32_t ch = cfirst; ch < c1; ch += cstep) {
    // WALK: the input sites of the lane's index at t - 1, t, t + 1
    Fetched<SF, 1> rp, rc, rn;
    for (int tt = 0; tt < a.tchunk; ++tt) {
        const uint32_t w = ch * blockDim.x + threadIdx.x;
        const bool valid = w < a.total;
        const uint32_t q = fdiv(w, a.div_groups);
        const uint32_t j = w - q * (uint32_t)a.groups;
        uint32_t i;
        if (a.tile_y > 0) {
            // q = (tile * nk + k) * tile_cols + col; col = xh + Lxh (yl + tile_y zl); the
            // lane walks t = k tchunk + tt (nk = Lt / tchunk time chunks per tile)
            const uint32_t rest = fdiv(q, a.div_tcols);
            const uint32_t col = q - rest * (uint32_t)(g.Lxh * a.tile_y * a.tile_z);
            const uint32_t tile = fdiv(rest, a.div_nk);
            const uint32_t kc = rest - tile * ((uint32_t)g.L[3] / (uint32_t)a.tchunk);
            const uint32_t t = kc * (uint32_t)a.tchunk + (uint32_t)tt;
            const uint32_t r1 = fdiv(col, a.div_lxh);
            const uint32_t xh = col - r1 * (uint32_t)g.Lxh;
            const uint32_t zl = fdiv(r1, a.div_ty);
            const uint32_t yl = r1 - zl * (uint32_t)a.tile_y;
            const uint32_t tz = fdiv(tile, a.div_nty);
            const uint32_t ty = tile - tz * (uint32_t)(g.L[1] / a.tile_y);
            const uint32_t y = ty * a.tile_y + yl, z = tz * a.tile_z + zl;
            i = xh + (uint32_t)g.Lxh * (y + (uint32_t)g.L[1] * z) + ncol * t;
        } else {
            const uint32_t k = fdiv(q, a.div_ncol);
            i = q + k * ncol * (uint32_t)(a.tchunk - 1) + (uint32_t)tt * ncol;
        }
        int x[4];
        site_coords(g, i, p, x);
        const uint32_t *staged = nullptr;
        const float *cstaged = nullptr;
        (void)cstaged;
        if constexpr (SHL) {
            // block = sites_per_block sites x groups lanes, whole sites; lane j stages links
            // j, j + groups, ... (link d: mu = d / 2, backward for odd d)
            const uint32_t slot = threadIdx.x / (uint32_t)a.groups;
            uint32_t *mine = stage + slot * kStageSite;
            __syncthreads();  // the previous site's links are no longer read
            for (uint32_t d = j; valid && d < 8; d += (uint32_t)a.groups) {
                const int mu = (int)(d >> 1);
                const uint32_t n = nb_bwd_rt(g, i, x, mu);
                stage_link<LF>(a.gauge, g.S, p, mu, (d & 1) != 0, i, n, mine + d * kStageWords);
            }
            if constexpr (SCL) {
                float *cm = cstage + slot * kClovStage;
                for (uint32_t m = j; valid && m < 36; m += (uint32_t)a.groups)
                    stage_clover_pair(a.clov, g.S, p, i, (int)m, cm);
                cstaged = cm;
            }
            __syncthreads();
            staged = mine;
        }
        if (!valid) continue;
        C acc[RPT][12];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[r][c] = {(T)0, (T)0};

        if constexpr (WALK) {
            // a step of the time walk: rp and rc carried over (loaded at the first step),
            // the x neighbour that is not site i and the y, z neighbours through f0 / rp,
            // rn (t + 1) loaded for this step and kept for the next two.  rn is loaded
            // after the y and z neighbours: those are the t sites that other lanes loaded
            // as their rn one step earlier, and issuing them first shortens the time such
            // a line has to stay in L2 (measured: 1.8 GB fewer reads per launch at 48^3 x 96)
            const bool bx = (x[0] & 1) != 0;  // x = 2 xh + bx: site i is the x neighbour
            Fetched<SF, 1> f0;
            if (tt == 0) {
                fetch_site<SF>(in, nb_bwd(g, i, x, 3), j, rp);
                fetch_site<SF>(in, i, j, rc);
            }
            fetch_site<SF>(in, bx ? nb_fwd(g, i, x, 0) : nb_bwd(g, i, x, 0), j, f0);
            hop_dir<3, 1, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, rp);
            fetch_site<SF>(in, nb_fwd(g, i, x, 1), j, rp);
            // in place: rc <- the forward x neighbour, f0 <- the backward one (undone below)
            auto swap_x = [&]() {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const auto u = f0.s[0][c], v = rc.s[0][c];
                    f0.s[0][c] = bx ? v : u;
                    rc.s[0][c] = bx ? u : v;
                }
                const float su = f0.scl[0], sv = rc.scl[0];
                f0.scl[0] = bx ? sv : su;
                rc.scl[0] = bx ? su : sv;
                const uint32_t nu = f0.n, nv = rc.n;
                f0.n = bx ? nv : nu;
                rc.n = bx ? nu : nv;
            };
            rc.n = i;
            swap_x();
            hop_dir<0, 0, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, rc);
            hop_dir<0, 1, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, f0);
            swap_x();
            fetch_site<SF>(in, nb_bwd(g, i, x, 1), j, f0);
            hop_dir<1, 0, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, rp);
            fetch_site<SF>(in, nb_fwd(g, i, x, 2), j, rp);
            hop_dir<1, 1, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, f0);
            fetch_site<SF>(in, nb_bwd(g, i, x, 2), j, f0);
            fetch_site<SF>(in, nb_fwd(g, i, x, 3), j, rn);
            hop_dir<2, 0, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, rp);
            hop_dir<2, 1, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, f0);
            hop_dir<3, 0, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, rn);
            // the next step's t - 1 and t sites (its t + 1 site follows t + 1 here)
            rp = rc;
            rc = rn;
        } else {
            // directions computed one behind their fetch (two buffers, A and B), in the
            // order hop_order
            constexpr int d0 = hop_order(0), d1 = hop_order(1), d2 = hop_order(2),
                          d3 = hop_order(3), d4 = hop_order(4), d5 = hop_order(5),
                          d6 = hop_order(6), d7 = hop_order(7);
            Fetched<SF, RPT> fa, fb;
            hop_fetch<d0 / 2, d0 % 2, SF, RPT>(a, in, i, x, j, fa);
            hop_fetch<d1 / 2, d1 % 2, SF, RPT>(a, in, i, x, j, fb);
            hop_dir<d0 / 2, d0 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fa);
            hop_fetch<d2 / 2, d2 % 2, SF, RPT>(a, in, i, x, j, fa);
            hop_dir<d1 / 2, d1 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fb);
            hop_fetch<d3 / 2, d3 % 2, SF, RPT>(a, in, i, x, j, fb);
            hop_dir<d2 / 2, d2 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fa);
            hop_fetch<d4 / 2, d4 % 2, SF, RPT>(a, in, i, x, j, fa);
            hop_dir<d3 / 2, d3 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fb);
            hop_fetch<d5 / 2, d5 % 2, SF, RPT>(a, in, i, x, j, fb);
            hop_dir<d4 / 2, d4 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fa);
            hop_fetch<d6 / 2, d6 % 2, SF, RPT>(a, in, i, x, j, fa);
            hop_dir<d5 / 2, d5 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fb);
            hop_fetch<d7 / 2, d7 % 2, SF, RPT>(a, in, i, x, j, fb);
            hop_dir<d6 / 2, d6 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fa);
            hop_dir<d7 / 2, d7 % 2, SF, LF, RPT, RPH, SHL, FL>(a, p, i, x, sg_f, acc, staged, fb);
        }

        const T ca = (T)a.a;
        constexpr bool CG = EPI == EPI_XPAY_CG || EPI == EPI_CLOV_XPAY_CG;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const uint32_t rr = j * RPT + r;
            C *o = acc[r];  // the epilogue result replaces the accumulator
            if constexpr (EPI == EPI_XPAY || EPI == EPI_XPAY_CG) {
                C xv[12];
                xin.load(i, rr, xv);
#pragma unroll
                for (int c = 0; c < 12; ++c) o[c] = add_s(xv[c], ca, o[c]);
            } else if constexpr (EPI == EPI_CLOV) {
                C d[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) d[c] = o[c];
                if constexpr (SCL)
                    clover_apply_lds<T>(cstaged, d, o);
                else
                    clover_apply<CR, T>(a.clov, g.S, p, i, d, o);
            } else if constexpr (EPI == EPI_CLOV_XPAY || EPI == EPI_CLOV_XPAY_CG) {
                C xv[12], cx[12];
                xin.load(i, rr, xv);
                if constexpr (SCL)
                    clover_apply_lds<T>(cstaged, xv, cx);
                else
                    clover_apply<CR, T>(a.clov, g.S, p, i, xv, cx);
#pragma unroll
                for (int c = 0; c < 12; ++c) o[c] = add_s(cx[c], ca, o[c]);
            } else if constexpr (EPI == EPI_XPAY_CLOV) {
                C xv[12];
                xin.load(i, rr, xv);
#pragma unroll
                for (int c = 0; c < 12; ++c) xv[c] = add_s(xv[c], ca, o[c]);
                if constexpr (SCL)
                    clover_apply_lds<T>(cstaged, xv, o);
                else
                    clover_apply<CR, T>(a.clov, g.S, p, i, xv, o);
            }
            if constexpr (CG) {
                // x += alpha p, r -= alpha o; o becomes the stored r (for the norm)
                const double den = a.cg_pi[rr] + (a.cg_pi2 ? a.cg_pi2[rr] : 0.0);
                const T al = (T)(a.cg_active[rr] && den != 0.0 ? a.cg_rho[rr] / den : 0.0);
                {
                    C xv[12], pv[12];
                    cgx.load(i, rr, xv);
                    cgp.load(i, rr, pv);
#pragma unroll
                    for (int c = 0; c < 12; ++c)
                        xv[c] = {fma(al, pv[c].x, xv[c].x), fma(al, pv[c].y, xv[c].y)};
                    cgx.store(i, rr, xv);
                }
                C rv[12];
                cgr.load(i, rr, rv);
#pragma unroll
                for (int c = 0; c < 12; ++c)
                    rv[c] = {fma(-al, o[c].x, rv[c].x), fma(-al, o[c].y, rv[c].y)};
                cgr.store(i, rr, rv);  // rv: now the stored (rounded) values
#pragma unroll
                for (int c = 0; c < 12; ++c) o[c] = rv[c];
            } else if constexpr (SF != SpinorFmt::F16) {
                out.store(i, rr, o);
            }
        }
        // FP16: one wide store per component for the lane's RPT right-hand sides;
        // acc then holds the stored (rounded) values
        if constexpr (SF == SpinorFmt::F16 && !CG)
            out.template store_group<RPT>(i, j * RPT, acc, a.want_norm != 0);
        if (a.want_norm) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 12; ++c) s += (double)norm2(acc[r][c]);
                nrm[r] += s;
            }
        }
    }
    }
    if (a.want_norm) {
        const int slot = threadIdx.x / a.groups;
        const int jj = threadIdx.x - slot * a.groups;
        block_sum_to_partial<RPT>(red, a.sites_per_block, a.nrhs, slot, jj * RPT, RPT, nrm,
                                  a.partial, blockIdx.x, gridDim.x);
    }
}

template <SpinorFmt SF, LinkFmt LF, typename CR, int RPT, int EPI, bool RPH, bool SHL,
          bool FL = false>
hipError_t hop_launch_t(const HopArgs &a, int grid, int block, hipStream_t st) {
    const size_t shm = a.want_norm ? (size_t)a.sites_per_block * a.nrhs * sizeof(double) : 0;
    if constexpr (hop_walks<SF, RPT, EPI, SHL, FL>()) {
        if (a.tchunk > 1) {
            if (a.occupancy)
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    a.occupancy, hop_kernel<SF, LF, CR, RPT, EPI, RPH, SHL, FL, true>, block,
                    shm);
            hipLaunchKernelGGL((hop_kernel<SF, LF, CR, RPT, EPI, RPH, SHL, FL, true>), dim3(grid),
                               dim3(block), shm, st, a);
            return hipGetLastError();
        }
    }
    if (a.occupancy)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            a.occupancy, hop_kernel<SF, LF, CR, RPT, EPI, RPH, SHL, FL>, block, shm);
    hipLaunchKernelGGL((hop_kernel<SF, LF, CR, RPT, EPI, RPH, SHL, FL>), dim3(grid), dim3(block),
                       shm, st, a);
    return hipGetLastError();
}

template <SpinorFmt SF, LinkFmt LF, typename CR, int RPT, bool RPH, bool SHL = false,
          bool FL = false>
hipError_t hop_launch_epi(const HopArgs &a, int grid, int block, hipStream_t st) {
    switch (a.epi) {
        case EPI_NONE:
            return hop_launch_t<SF, LF, CR, RPT, EPI_NONE, RPH, SHL, FL>(a, grid, block, st);
        case EPI_XPAY:
            return hop_launch_t<SF, LF, CR, RPT, EPI_XPAY, RPH, SHL, FL>(a, grid, block, st);
        case EPI_CLOV:
            return hop_launch_t<SF, LF, CR, RPT, EPI_CLOV, RPH, SHL, FL>(a, grid, block, st);
        case EPI_CLOV_XPAY:
            return hop_launch_t<SF, LF, CR, RPT, EPI_CLOV_XPAY, RPH, SHL, FL>(a, grid, block, st);
        case EPI_XPAY_CLOV:
            return hop_launch_t<SF, LF, CR, RPT, EPI_XPAY_CLOV, RPH, SHL, FL>(a, grid, block, st);
        case EPI_XPAY_CG:
            return hop_launch_t<SF, LF, CR, RPT, EPI_XPAY_CG, RPH, SHL, FL>(a, grid, block, st);
        case EPI_CLOV_XPAY_CG:
            return hop_launch_t<SF, LF, CR, RPT, EPI_CLOV_XPAY_CG, RPH, SHL, FL>(a, grid, block,
                                                                               st);
    }
    return hipErrorInvalidValue;
}

// The FLIC hop (thin links a.gauge, fat links a.gauge_fat, both in format LF): one rhs
// per lane, links loaded per lane.
template <SpinorFmt SF, LinkFmt LF, typename CR>
hipError_t hop_launch_flic_fmt(const HopArgs &a, int rpt, int grid, int block, hipStream_t st) {
    if (rpt != 1 || a.stage_links || !a.gauge_fat) return hipErrorInvalidValue;
    bool real_phase = true;
    for (int mu = 0; mu < 4; ++mu) real_phase &= a.phase[mu].y == 0.0;
    if (real_phase) return hop_launch_epi<SF, LF, CR, 1, true, false, true>(a, grid, block, st);
    return hop_launch_epi<SF, LF, CR, 1, false, false, true>(a, grid, block, st);
}

template <SpinorFmt SF, LinkFmt LF, typename CR>
hipError_t hop_launch_fmt(const HopArgs &a, int rpt, int grid, int block, hipStream_t st) {
    bool real_phase = true;
    for (int mu = 0; mu < 4; ++mu) real_phase &= a.phase[mu].y == 0.0;
    // several rhs per lane only where the accumulators fit (FP64 keeps one)
    constexpr bool multi = SF != SpinorFmt::F64;
    // links staged in LDS by the site's lanes: 12-real FP16 / FP32 links, one or two rhs
    // per lane
    constexpr bool stageable = LF == LinkFmt::F16_12 || LF == LinkFmt::F32_12;
    if constexpr (stageable) {
        if (a.stage_links && rpt == 1) {
            if (real_phase) return hop_launch_epi<SF, LF, CR, 1, true, true>(a, grid, block, st);
            return hop_launch_epi<SF, LF, CR, 1, false, true>(a, grid, block, st);
        }
        if (a.stage_links && rpt == 2) {
            if (real_phase) return hop_launch_epi<SF, LF, CR, 2, true, true>(a, grid, block, st);
            return hop_launch_epi<SF, LF, CR, 2, false, true>(a, grid, block, st);
        }
    }
    if (a.stage_links) return hipErrorInvalidValue;
    if (real_phase) {
        if (rpt == 1) return hop_launch_epi<SF, LF, CR, 1, true>(a, grid, block, st);
        if constexpr (multi) {
            if (rpt == 2) return hop_launch_epi<SF, LF, CR, 2, true>(a, grid, block, st);
            if (rpt == 3) return hop_launch_epi<SF, LF, CR, 3, true>(a, grid, block, st);
            if (rpt == 4) return hop_launch_epi<SF, LF, CR, 4, true>(a, grid, block, st);
        }
    } else {
        if (rpt == 1) return hop_launch_epi<SF, LF, CR, 1, false>(a, grid, block, st);
        if constexpr (multi) {
            if (rpt == 2) return hop_launch_epi<SF, LF, CR, 2, false>(a, grid, block, st);
            if (rpt == 3) return hop_launch_epi<SF, LF, CR, 3, false>(a, grid, block, st);
            if (rpt == 4) return hop_launch_epi<SF, LF, CR, 4, false>(a, grid, block, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace cola
