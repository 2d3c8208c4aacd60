// Library handle and host-side helpers shared by the C ABI, the operator
// composition and the solvers.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/cola.h"
#include "common.h"
#include "launch.h"

namespace cola {

constexpr int kMaxRhs = kRedMaxWidth;
constexpr int kMaxGrid = kRedMaxBlocks;
constexpr int kEigMax = 32;  // eigenpairs of one cola_eigensolve call
// size of the fixed device workspace of cola_dslash_apply_noalloc (per device)
constexpr size_t kScratchBytes = (size_t)128 << 20;

struct TuneEntry {
    int rpt = 1;
    int sites_per_block = 64;
    int grid = 0;    // 0: one block per sites_per_block site columns; -1: the blocks
                     // resident at once (grid-stride loop, no tail of late blocks)
    int tchunk = 1;  // timeslices walked by one lane
    int tile_y = 0;  // spatial tile (all x-rows x tile_y x tile_z); 0 = lexicographic
    int tile_z = 0;
    int stage = 0;   // links staged in LDS by the lanes of a site (see stage_ok)
    double ms = 0;
};

// A pool of device vectors keyed by a small integer tag (kept until destroy).
struct VecCache {
    std::map<std::string, std::pair<void *, size_t>> bufs;
};

}  // namespace cola

struct cola_handle {
    int dims[4];
    cola::Geom g;
    double kappa = 0, csw = 0;
    cola::Cplx64 phase[4];
    unsigned flags = 0;
    int device = 0;
    int num_cu = 0;  // compute units of the device
    std::string arch;  // the device's architecture name (tuned shapes are kept per device)
    std::map<std::string, int> occupancy;  // resident blocks per CU by launch variant

    // packed gauge fields by cola::LinkFmt
    void *gauge[4] = {nullptr, nullptr, nullptr, nullptr};
    bool gauge_set = false;
    bool su3 = false;
    double su3_dev = 0;
    // FLIC operator: the smeared ("fat") links in the packed formats of `gauge`; flic is
    // set by cola_set_fat_gauge and cleared by cola_set_gauge
    void *fat[4] = {nullptr, nullptr, nullptr, nullptr};
    bool flic = false;
    // clover blocks (both parities): A and A^-1, FP64 and FP32
    void *clov64 = nullptr, *clovinv64 = nullptr, *clov32 = nullptr, *clovinv32 = nullptr;

    // reductions
    double *partial = nullptr;  // kRedPartialDoubles (block, then group partials)
    unsigned *counter = nullptr;  // kRedCounters tickets, left at 0 between launches
    double *scal = nullptr;  // scalar arrays, kScalSlots * kMaxRhs
    int *active = nullptr;   // kMaxRhs
    double *host_scal = nullptr;  // pinned mirror of scal
    int *host_active = nullptr;   // pinned

    cola::VecCache cache;
    std::string err;

    // timing of hop launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<double> pending_bytes, pending_flops;
    std::vector<int> pending_prec, pending_epi;
    std::vector<hipEvent_t> event_pool;
    cola_stats_t stats{};

    // device address of this device's fixed workspace (cola_dslash_apply_noalloc)
    void *scratch = nullptr;

    // autotuning
    int tune_mode = 0;
    std::map<std::string, cola::TuneEntry> tune;

    // CG iteration blocks of small solves captured as HIP graphs, by everything their
    // launches bake in (vectors, fields, shape); a side stream for capture and replay
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t gstream = nullptr;
    hipEvent_t gevent = nullptr;
};

namespace cola {

constexpr int kScalSlots = 16;

int set_error(cola_handle_t *h, int code, const std::string &msg);
// drops the captured graphs (their launches hold workspace addresses)
void graphs_clear(cola_handle_t *h);
int hip_error(cola_handle_t *h, hipError_t e, const char *what);

#define COLA_HIP(h, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::cola::hip_error((h), e_, #call); \
    } while (0)
#define COLA_TRY(call)                \
    do {                              \
        int rc_ = (call);             \
        if (rc_ < 0) return rc_;      \
    } while (0)

SpinorFmt spinor_fmt(int prec);
LinkFmt link_fmt(int prec);
size_t spinor_block_bytes(const Geom &g, SpinorFmt f, int nrhs);

// device vector from the handle's cache (zero-filled on first allocation)
int get_vec(cola_handle_t *h, const std::string &tag, size_t bytes, void **out);

// the reduction target writing into scalar slot `slot`
Reduce reduce_into(cola_handle_t *h, int slot);
inline double *scal_slot(cola_handle_t *h, int slot) { return h->scal + slot * kMaxRhs; }

// one half-lattice hop launch with epilogue
struct HopCall {
    void *out;
    const void *in;
    int parity;
    int dagger;
    int epi = EPI_NONE;
    const void *x = nullptr;
    double a = 0;
    const void *clov = nullptr;
    double *norm_result = nullptr;  // per-rhs |out|^2 (fused)
    // EPI_XPAY_CG / EPI_CLOV_XPAY_CG: the CG vectors and per-rhs scalars
    void *cg_x = nullptr, *cg_r = nullptr;
    const void *cg_p = nullptr;
    const double *cg_rho = nullptr, *cg_pi = nullptr, *cg_pi2 = nullptr;
    const int *cg_active = nullptr;
    // fixed: no launch-shape tuning, no timing events, no occupancy queries (the
    // non-allocating entry point); the shape is the cached or the default one
    bool fixed = false;
};
int hop(cola_handle_t *h, const HopCall &c, int prec, int nrhs, hipStream_t st);

// One CG step on the even-odd normal system S^dag S, with the update fused into the
// last hop: pi = |S p|^2, then with alpha = rho / pi per active rhs,
//   x += alpha p,  r -= alpha S^dag S p,  rho_new = |r|^2.
// x, r, p: even-parity blocks in the storage of prec.
int schur_normal_cg_step(cola_handle_t *h, int prec, int nrhs, hipStream_t st, void *x, void *r,
                         const void *p, const double *rho, double *pi, const int *active,
                         double *rho_new);

// composite operators on packed fields (see COLA_OP_*); norm_result (optional)
// receives |out|^2 per rhs where the composition allows it to be fused.  ws: a
// caller-provided workspace of op_workspace_bytes() for the intermediate vectors
// (the hops then run in their fixed shapes, untimed); nullptr: the handle's cache.
int apply_op(cola_handle_t *h, void *out, const void *in, int op, int parity, int prec, int nrhs,
             hipStream_t st, double *norm_result = nullptr, char *ws = nullptr);
size_t op_workspace_bytes(const cola_handle_t *h, int op, int prec, int nrhs);

// low-eigenmode solver and deflated CG (eigen.cpp)
int eigensolve_impl(cola_handle_t *h, void *X, int n, const cola_eig_params_t *p,
                    cola_eig_result_t *r, hipStream_t st);
int cg_deflated_impl(cola_handle_t *h, void *x, const void *b, int nrhs, const void *X,
                     const double *lambda, int n, const cola_cg_params_t *p, cola_cg_result_t *r,
                     hipStream_t st);

// device address of this handle's device's fixed workspace (kScratchBytes)
int scratch_address(cola_handle_t *h, void **out);

// timing bookkeeping
int flush_timing(cola_handle_t *h, bool wait_all);

std::string tune_key(const cola_handle_t *h, int prec, int nrhs, int epi, int norm);
// the process-wide table of tuned launch shapes and its file (path null: the default
// file); return the number of entries read / written, or < 0
int tune_cache_load(cola_handle_t *h, const char *path);
int tune_cache_save(cola_handle_t *h, const char *path);

}  // namespace cola
