// Internal definitions shared by the HIP kernels and the host library.
//
// Packed (library-internal) layouts, all per parity p (0 even, 1 odd):
//   checkerboard index i of a site of parity p: i = (x + Lx*(y + Ly*(z + Lz*t))) / 2,
//   0 <= i < Vh = V/2; arrays are padded to a stride S = Vh rounded up to 64.
//   spinor block (one parity, R right-hand sides): complex element of spin-colour
//     component c (= 3*spin + colour), site i, rhs r at ((c*S + i)*R + r); for FP16
//     the block continues with one float scale per (i, r) at index i*R + r.
//     A full-lattice field is the even block followed by the odd block.
//   gauge (one precision): chunk k of link U_mu at site i of parity p at
//     ((p*4 + mu)*NCH + k)*S + i, NCH chunks of 16 bytes (8 for FP16).
//   clover (one precision): real pair k (0..35) of site i, parity p at (p*36 + k)*S + i;
//     two Hermitian 6x6 chiral blocks, each 6 diagonal reals then the 15 complex
//     entries below the diagonal, row-major.
#pragma once

#include <stdint.h>

namespace cola {

constexpr int kStrideAlign = 64;

// Per-parity stride of the packed fields: the checkerboard volume rounded up to an odd
// multiple of 64 sites.  With power-of-two lattice extents an even multiple starts the
// component arrays (c * S * R apart) at addresses sharing many low bits, and the 24 loads
// of one lane then pile onto the same cache sets and memory channels (the odd stride made
// the hops 2.5-9% faster at 48^3 x 96 and 32^3 x 64).
inline int packed_stride(int vh) {
    int s = (vh + kStrideAlign - 1) / kStrideAlign * kStrideAlign;
    if ((s / kStrideAlign) % 2 == 0) s += kStrideAlign;
    return s;
}

// Division by a runtime-constant divisor with a multiply-high and a shift
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994).  Exact for numerators below 2^31.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
    return f;
}

struct Geom {
    int L[4];        // Lx, Ly, Lz, Lt
    int Lxh;         // Lx / 2
    int Vh;          // sites of one parity
    int S;           // padded per-parity stride
    int s1, s2, s3;  // checkerboard strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
    FastDiv div_xh, div_y, div_z;
};

enum class SpinorFmt : int { F64 = 0, F32 = 1, F16 = 2 };
enum class LinkFmt : int { F64_18 = 0, F64_12 = 1, F32_12 = 2, F16_12 = 3 };

enum Epilogue : int {
    EPI_NONE = 0,        // out = D in
    EPI_XPAY = 1,        // out = x + a D in
    EPI_CLOV = 2,        // out = C (D in)              C: clover blocks of the output parity
    EPI_CLOV_XPAY = 3,   // out = C x + a D in
    EPI_XPAY_CLOV = 4,   // out = C (x + a D in)
    // CG step fused into the last hop of the normal operator: with o = x + a D in
    // (EPI_XPAY_CG) or C x + a D in (EPI_CLOV_XPAY_CG), and per rhs
    // alpha = active ? rho / (pi + pi2) : 0:  cg_x += alpha cg_p,  cg_r -= alpha o;
    // o itself is not stored and the fused norm is |cg_r|^2
    EPI_XPAY_CG = 5,
    EPI_CLOV_XPAY_CG = 6
};

struct Cplx64 {
    double x, y;
};

struct HopArgs {
    Geom g;
    int parity;      // output parity
    int dagger;      // 0: D, 1: D^H
    int nrhs;        // R
    int groups;      // R / rhs-per-thread
    FastDiv div_groups;
    int epi;         // Epilogue
    int want_norm;   // per-block partials of |out|^2 per rhs into `partial`
    double a;        // epilogue coefficient
    Cplx64 phase[4]; // boundary phases e^{i theta_mu}
    const void *in;      // parity (1 - parity) block
    void *out;           // parity `parity` block
    const void *x;       // parity `parity` block (epilogues 1, 3, 4)
    const void *gauge;   // packed gauge buffer of the launch precision
    const void *gauge_fat;  // FLIC operator: packed smeared links (same format), else null
    const void *clov;    // packed clover buffer (both parities) for epilogues 2-4
    double *partial;     // per-block |out|^2 partials [R][grid] (want_norm)
    uint32_t total;      // (Lt / tchunk) * (Vh / Lt) * groups lanes of work
    int sites_per_block; // T: threads per block = T * groups
    int tchunk;          // timeslices one lane walks (t-streaming); divides Lt
    FastDiv div_ncol;    // division by the checkerboard sites of one timeslice
    // spatial tiling (tile_y > 0): work ordered (tile, time chunk, column in tile); a
    // tile is all x-rows of tile_y x tile_z (y, z) columns; div_nk divides by the time
    // chunks Lt / tchunk
    int tile_y, tile_z;
    FastDiv div_tcols, div_nk, div_lxh, div_ty, div_nty;
    // the site's links staged in LDS by its first eight lanes (groups >= 8, one rhs per
    // lane, sites_per_block <= 32, 12-real FP16 / FP32 links)
    int stage_links;
    // host only: when set, the launcher stores the kernel's resident blocks per CU here
    // instead of launching
    int *occupancy;
    // CG epilogues: the solver's vectors (parity `parity` blocks of the launch format)
    // and its per-rhs scalars
    void *cg_x, *cg_r;
    const void *cg_p;
    const double *cg_rho, *cg_pi, *cg_pi2;
    const int *cg_active;
};

// Deterministic reductions.  Kernels write per-block partial sums, column-major
// (partial[q * nblocks + b], at most kRedMaxBlocks blocks of kRedMaxWidth columns), and a
// reduce launch adds them in block order.  The block-CG Gram kernel (few blocks, wide
// rows) instead sums per group of kRedGroup blocks with atomic tickets, then over the
// groups; its block rows and group rows fit the same array, and the counter array holds
// one ticket per group and one for the groups.
constexpr int kRedGroup = 256;
constexpr int kRedMaxBlocks = 65536;
constexpr int kRedMaxWidth = 16;
constexpr int kRedGroups = kRedMaxBlocks / kRedGroup;
constexpr size_t kRedPartialDoubles = (size_t)(kRedMaxBlocks + kRedGroups) * kRedMaxWidth;
constexpr int kRedCounters = kRedGroups + 1;

// Sites of one block when the hop stages each site's links in LDS.
constexpr int kStageSites = 32;

// Link chunk counts per format.
constexpr int link_chunks(LinkFmt f) {
    return f == LinkFmt::F64_18 ? 9 : f == LinkFmt::F64_12 ? 6 : 3;
}
constexpr int link_chunk_bytes(LinkFmt f) { return f == LinkFmt::F16_12 ? 8 : 16; }
constexpr int link_reals(LinkFmt f) { return f == LinkFmt::F64_18 ? 18 : 12; }
constexpr int link_real_bytes(LinkFmt f) {
    return f == LinkFmt::F16_12 ? 2 : f == LinkFmt::F32_12 ? 4 : 8;
}
constexpr int spinor_real_bytes(SpinorFmt f) {
    return f == SpinorFmt::F64 ? 8 : f == SpinorFmt::F32 ? 4 : 2;
}

}  // namespace cola
