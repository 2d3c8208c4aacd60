// Host side of the operators: hop launches (with launch-shape tuning and
// optional event timing), composition of M, M^H, M^H M and the even-site
// Schur complement from half-lattice hops, and small handle utilities.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include <sys/stat.h>
#include <unistd.h>

#include "handle.h"

namespace cola {

int set_error(cola_handle_t *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

int hip_error(cola_handle_t *h, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(h, e == hipErrorOutOfMemory ? COLA_ENOMEM : COLA_EHIP, m);
}

SpinorFmt spinor_fmt(int prec) {
    switch (prec) {
        case COLA_FP64:
        case COLA_FP64_12: return SpinorFmt::F64;
        case COLA_FP32: return SpinorFmt::F32;
        default: return SpinorFmt::F16;
    }
}

LinkFmt link_fmt(int prec) {
    switch (prec) {
        case COLA_FP64: return LinkFmt::F64_18;
        case COLA_FP64_12: return LinkFmt::F64_12;
        case COLA_FP32: return LinkFmt::F32_12;
        default: return LinkFmt::F16_12;
    }
}

size_t spinor_block_bytes(const Geom &g, SpinorFmt f, int nrhs) {
    const size_t SR = (size_t)g.S * nrhs;
    switch (f) {
        case SpinorFmt::F64: return 12 * SR * 16;
        case SpinorFmt::F32: return 12 * SR * 8;
        default: return 12 * SR * 4 + SR * 4;
    }
}

int get_vec(cola_handle_t *h, const std::string &tag, size_t bytes, void **out) {
    auto it = h->cache.bufs.find(tag);
    if (it != h->cache.bufs.end() && it->second.second >= bytes) {
        *out = it->second.first;
        return COLA_OK;
    }
    if (it != h->cache.bufs.end()) {
        COLA_HIP(h, hipDeviceSynchronize());
        graphs_clear(h);  // captured launches may hold the old address
        COLA_HIP(h, hipFree(it->second.first));
        h->cache.bufs.erase(it);
    }
    void *p = nullptr;
    COLA_HIP(h, hipMalloc(&p, bytes));
    COLA_HIP(h, hipMemset(p, 0, bytes));
    h->cache.bufs[tag] = {p, bytes};
    *out = p;
    return COLA_OK;
}

Reduce reduce_into(cola_handle_t *h, int slot) {
    return Reduce{h->partial, h->counter, scal_slot(h, slot)};
}

// The file of tuned shapes: $COLA_TUNE_CACHE (empty: none), else
// $XDG_CACHE_HOME/cola/hop_tune.txt or ~/.cache/cola/hop_tune.txt.
std::string tune_cache_path() {
    if (const char *p = getenv("COLA_TUNE_CACHE")) return p;
    if (const char *x = getenv("XDG_CACHE_HOME"))
        if (x[0]) return std::string(x) + "/cola/hop_tune.txt";
    if (const char *hm = getenv("HOME"))
        if (hm[0]) return std::string(hm) + "/.cache/cola/hop_tune.txt";
    return "";
}

std::string tune_key(const cola_handle_t *h, int prec, int nrhs, int epi, int norm) {
    char buf[160];
    snprintf(buf, sizeof buf, "hop:%dx%dx%dx%d:p%d:r%d:e%d:n%d", h->dims[0], h->dims[1],
             h->dims[2], h->dims[3], prec, nrhs, epi, norm);
    return buf;
}

namespace {

int spinor_site_bytes(SpinorFmt f) { return f == SpinorFmt::F64 ? 192 : f == SpinorFmt::F32 ? 96 : 52; }
int link_bytes(LinkFmt f) { return link_chunks(f) * link_chunk_bytes(f); }

void hop_work(const cola_handle_t *h, int prec, int nrhs, int epi, double *bytes, double *flops) {
    const SpinorFmt sf = spinor_fmt(prec);
    const LinkFmt lf = link_fmt(prec);
    const double Vh = h->g.Vh;
    // FLIC: the thin and the smeared link of each direction, two projections and four
    // SU(3) products (twice the Wilson count) plus 36 flops to combine the links
    const double nl = h->flic ? 2.0 : 1.0;
    double b = 8.0 * nl * link_bytes(lf) + 2.0 * nrhs * spinor_site_bytes(sf);
    double f = nl * 1320.0 * nrhs + nl * (lf == LinkFmt::F64_18 ? 0.0 : 8 * 42.0) +
               (h->flic ? 8 * 36.0 : 0.0);
    const bool cg = epi == EPI_XPAY_CG || epi == EPI_CLOV_XPAY_CG;
    if (epi == EPI_XPAY || epi == EPI_CLOV_XPAY || epi == EPI_XPAY_CLOV || cg) {
        b += nrhs * spinor_site_bytes(sf);
        f += 48.0 * nrhs;
    }
    if (cg) {
        // reads x, p, r and writes x, r in place of writing the result
        b += 4.0 * nrhs * spinor_site_bytes(sf);
        f += 96.0 * nrhs;
    }
    if (epi == EPI_CLOV || epi == EPI_CLOV_XPAY || epi == EPI_XPAY_CLOV ||
        epi == EPI_CLOV_XPAY_CG) {
        b += 72.0 * (sf == SpinorFmt::F64 ? 8 : 4);
        f += 552.0 * nrhs;
    }
    *bytes = b * Vh;
    *flops = f * Vh;
}

hipEvent_t take_event(cola_handle_t *h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch shape for one hop launch: T site columns x groups lanes per block.
void shape_for(const TuneEntry &t, int Vh, int nrhs, int *groups, int *T, int *grid, int *block) {
    *groups = nrhs / t.rpt;
    *T = t.sites_per_block;
    *block = *T * *groups;
    const long cols = Vh / t.tchunk;
    long g = (cols + *T - 1) / *T;
    if (t.grid > 0 && t.grid < g) g = t.grid;  // t.grid < 0: resident cap applied later
    if (g > kMaxGrid) g = kMaxGrid;
    *grid = (int)std::max(1L, g);
}

// Longest power-of-two time chunk (<= 16, dividing Lt) that still leaves about
// 2^18 lanes of work, so a lattice fills the 256 CUs.
int default_tchunk(const Geom &g, int groups) {
    int tc = 1;
    while (tc * 2 <= 16 && g.L[3] % (tc * 2) == 0 &&
           (double)g.Vh * groups / (tc * 2) >= 262144.0)
        tc *= 2;
    return tc;
}

// A spatial tile must divide the y and z extents (tile_y = 0: no tiling).
bool tile_ok(const Geom &g, int ty, int tz) {
    if (ty == 0 && tz == 0) return true;
    return ty > 0 && tz > 0 && g.L[1] % ty == 0 && g.L[2] % tz == 0;
}

// Link staging: one or two rhs per lane, at least three lanes per site to share the
// eight links, whole sites of at most kStageSites per block, a 12-real FP16 or FP32 field
// and a packed field addressable with 32-bit byte offsets.
bool stage_ok(const Geom &g, int prec, int nrhs, const TuneEntry &t) {
    if (prec != COLA_FP16 && prec != COLA_FP32) return false;
    const double bytes = 8.0 * 3 * g.S * (prec == COLA_FP16 ? 8 : 16);
    return (t.rpt == 1 || t.rpt == 2) && nrhs / t.rpt >= 3 && t.sites_per_block <= kStageSites &&
           bytes < 2147483648.0;
}

// A launch shape the hop kernels accept for this lattice, precision and rhs count.
bool shape_valid(const Geom &g, int prec, int nrhs, const TuneEntry &e) {
    const bool f64 = prec == COLA_FP64 || prec == COLA_FP64_12;
    return (e.rpt >= 1 && e.rpt <= 4) && nrhs % e.rpt == 0 && (e.rpt == 1 || !f64) &&
           e.sites_per_block >= 1 && (e.sites_per_block & (e.sites_per_block - 1)) == 0 &&
           e.sites_per_block * (nrhs / e.rpt) <= 256 && e.grid >= -1 && e.tchunk >= 1 &&
           g.L[3] % e.tchunk == 0 && tile_ok(g, e.tile_y, e.tile_z);
}

// ---- the persistent table of tuned shapes
// Shared by every handle of the process and kept in a text file (one entry per line:
// device tag, key, rpt, sites per block, grid, time chunk, tile y, tile z, staging, ms),
// so that shapes tuned once are used by default afterwards, in this process and later
// ones.  Every shape gives bitwise the same result, so a stale entry can only cost
// time; entries that do not fit the launch are ignored.
struct TuneStore {
    std::mutex mu;
    std::map<std::string, TuneEntry> table;
    bool loaded = false;
};

TuneStore &tune_store() {
    static TuneStore s;
    return s;
}

std::string store_key(const cola_handle_t *h, const std::string &key) {
    return h->arch + ":" + std::to_string(h->num_cu) + " " + key;
}

int read_table(const std::string &path, std::map<std::string, TuneEntry> &out) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return -1;
    char dev[128], key[160];
    TuneEntry e;
    int n = 0;
    while (fscanf(f, "%127s %159s %d %d %d %d %d %d %d %lf", dev, key, &e.rpt, &e.sites_per_block,
                  &e.grid, &e.tchunk, &e.tile_y, &e.tile_z, &e.stage, &e.ms) == 10) {
        out[std::string(dev) + " " + key] = e;
        ++n;
    }
    fclose(f);
    return n;
}

int write_table(const std::string &path, const std::map<std::string, TuneEntry> &t) {
    const size_t cut = path.find_last_of('/');
    if (cut != std::string::npos && cut > 0) {
        // create the directory chain (mkdir -p)
        for (size_t k = 1; k <= cut; ++k)
            if (k == cut || path[k] == '/') mkdir(path.substr(0, k).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return -1;
    for (const auto &kv : t) {
        const TuneEntry &e = kv.second;
        fprintf(f, "%s %d %d %d %d %d %d %d %.6f\n", kv.first.c_str(), e.rpt, e.sites_per_block,
                e.grid, e.tchunk, e.tile_y, e.tile_z, e.stage, e.ms);
    }
    if (fclose(f) != 0) return -1;
    return rename(tmp.c_str(), path.c_str()) == 0 ? (int)t.size() : -1;
}

TuneEntry default_entry(const Geom &g, int prec, int nrhs) {
    TuneEntry t;
    t.rpt = 1;
    const int G = nrhs;
    int T = 1;
    while (T * 2 * G <= 256) T *= 2;
    t.sites_per_block = T;
    t.grid = 0;
    t.tchunk = default_tchunk(g, G);
    // Spatial tiles ((y, z) columns walked through t).  Multi-rhs hops: the largest of
    // 8x8, 8x4 and 4x4 whose timeslice holds at most 1024 sites (Lx/2 ty tz), so that a
    // few timeslices of a tile stay in one XCD's L2 while it walks t.  Measured: 8x8 on
    // 32^3 x 64 gave the fastest 12-rhs FP16 solve (8x4 and 4x8 0.4-1.6% slower, 4x4 4%);
    // on 48^3 x 96, 8x4 and 4x4 ran the 12-rhs FP32 clover solve 9-10% faster than 16x8.
    // Lattices no candidate divides keep the time-chunk order.
    int ty = 0, tz = 0;
    const bool f64 = prec == COLA_FP64 || prec == COLA_FP64_12;
    if (nrhs >= 4) {
        const int cand[3][2] = {{8, 8}, {8, 4}, {4, 4}};
        for (const auto &c : cand) {
            if (g.Lxh * c[0] * c[1] <= 1024 && tile_ok(g, c[0], c[1])) {
                ty = c[0];
                tz = c[1];
                break;
            }
        }
    }
    // single-rhs hops: the tuner's picks on 32^3 x 64 (16x16 tiles of 64-site blocks for
    // FP64, 16x8 tiles for FP16, plain order in 128-site blocks for FP32)
    if (nrhs == 1 && f64) ty = 16, tz = 16, t.sites_per_block = 64;
    if (nrhs == 1 && prec == COLA_FP16) ty = 16, tz = 8;
    if (nrhs == 1 && prec == COLA_FP32) t.tchunk = 1, t.sites_per_block = 128;
    if (ty > 0 && tile_ok(g, ty, tz)) {
        t.tile_y = ty;
        t.tile_z = tz;
        t.tchunk = 1;
    }
    t.stage = nrhs >= 8 && stage_ok(g, prec, nrhs, t) ? 1 : 0;
    // FP32 and FP16 with staged links walk time with the neighbours of the lane's index
    // in registers: tiles walked in chunks of up to 8 timeslices.  Measured on the
    // 48^3 x 96 12-rhs FP32 clover hop: 8x8 and 16x4 tiles in 8-slice chunks ran 12%
    // faster than the best shape without the walk, 4x4 and 8x4 tiles 5-6%; on 32^3 x 64
    // FP16 the plain hop 7% faster.
    if ((prec == COLA_FP32 || prec == COLA_FP16) && t.stage && t.rpt == 1) {
        const int wt[4][2] = {{8, 8}, {16, 4}, {8, 4}, {4, 4}};
        for (const auto &c : wt) {
            if (!tile_ok(g, c[0], c[1])) continue;
            int tc = 8;
            while (g.L[3] % tc) tc /= 2;
            t.tile_y = c[0];
            t.tile_z = c[1];
            t.tchunk = tc;
            break;
        }
    }
    // Measurement knob: COLA_HOP_SHAPE="rpt,sites_per_block,grid,tchunk" pins the
    // untuned launch shape (ignored unless every field is valid for this launch).
    if (const char *env = getenv("COLA_HOP_SHAPE")) {
        TuneEntry e;
        e.stage = -1;
        const int n = sscanf(env, "%d,%d,%d,%d,%d,%d,%d", &e.rpt, &e.sites_per_block, &e.grid,
                             &e.tchunk, &e.tile_y, &e.tile_z, &e.stage);
        if ((n == 4 || n == 6 || n == 7) && shape_valid(g, prec, nrhs, e)) {
            // staging as asked where possible, else the default rule
            const bool ok = stage_ok(g, prec, nrhs, e);
            e.stage = e.stage < 0 ? (ok ? 1 : 0) : (e.stage && ok ? 1 : 0);
            t = e;
        }
    }
    return t;
}

// One hop launch in shape te; with a norm, the partial-sum reduction follows unless
// reduce is false (the caller then launches it, after its timing event).
int fill_and_launch(cola_handle_t *h, const HopCall &c, int prec, int nrhs, const TuneEntry &te,
                    hipStream_t st, bool reduce = true, int *grid_out = nullptr) {
    HopArgs a;
    memset(&a, 0, sizeof a);
    a.g = h->g;
    a.parity = c.parity;
    a.dagger = c.dagger;
    a.nrhs = nrhs;
    int groups, T, grid, block;
    shape_for(te, h->g.Vh, nrhs, &groups, &T, &grid, &block);
    a.groups = groups;
    a.div_groups = make_fastdiv((uint32_t)groups);
    a.epi = c.epi;
    a.want_norm = c.norm_result != nullptr;
    a.a = c.a;
    for (int mu = 0; mu < 4; ++mu) a.phase[mu] = h->phase[mu];
    a.in = c.in;
    a.out = c.out;
    a.x = c.x;
    a.cg_x = c.cg_x;
    a.cg_r = c.cg_r;
    a.cg_p = c.cg_p;
    a.cg_rho = c.cg_rho;
    a.cg_pi = c.cg_pi;
    a.cg_pi2 = c.cg_pi2;
    a.cg_active = c.cg_active;
    a.gauge = h->gauge[(int)link_fmt(prec)];
    a.gauge_fat = h->flic ? h->fat[(int)link_fmt(prec)] : nullptr;
    a.clov = c.clov;
    a.partial = h->partial;
    a.total = (uint32_t)(h->g.Vh / te.tchunk) * (uint32_t)groups;
    a.sites_per_block = T;
    a.tchunk = te.tchunk;
    a.div_ncol = make_fastdiv((uint32_t)h->g.s3);
    a.tile_y = te.tile_y;
    a.tile_z = te.tile_z;
    a.stage_links = te.stage;
    if (te.tile_y > 0) {
        const Geom &g = h->g;
        a.div_tcols = make_fastdiv((uint32_t)(g.Lxh * te.tile_y * te.tile_z));
        a.div_nk = make_fastdiv((uint32_t)(g.L[3] / te.tchunk));
        a.div_lxh = make_fastdiv((uint32_t)g.Lxh);
        a.div_ty = make_fastdiv((uint32_t)te.tile_y);
        a.div_nty = make_fastdiv((uint32_t)(g.L[1] / te.tile_y));
    }
    // Resident grids (te.grid < 0): the number of blocks the device holds at once, the
    // work in a grid-stride loop.
    if (te.grid < 0) {
        char key[96];
        bool rph = true;
        for (int mu = 0; mu < 4; ++mu) rph &= h->phase[mu].y == 0.0;
        snprintf(key, sizeof key, "%d:%d:%d:%d:%d:%d:%d:%d", prec, te.rpt, c.epi, a.want_norm,
                 te.stage, block, nrhs, (int)rph);
        auto it = h->occupancy.find(key);
        int occ = 0;
        if (it != h->occupancy.end()) {
            occ = it->second;
        } else {
            a.occupancy = &occ;
            COLA_HIP(h, launch_hop(a, link_fmt(prec), te.rpt, grid, block, st));
            a.occupancy = nullptr;
            h->occupancy[key] = occ;
        }
        const long cap = (long)std::max(1, occ) * std::max(1, h->num_cu);
        if (grid > cap) grid = (int)cap;
    }
    COLA_HIP(h, launch_hop(a, link_fmt(prec), te.rpt, grid, block, st));
    if (grid_out) *grid_out = grid;
    if (c.norm_result && reduce)
        COLA_HIP(h, launch_reduce_partials(h->partial, grid, nrhs, c.norm_result, st));
    return COLA_OK;
}

// The stored shape for this key, unless a shape is pinned by COLA_HOP_SHAPE or the entry
// does not fit this launch; load: read the file once per process if not yet read.
bool stored_entry(cola_handle_t *h, const std::string &key, int prec, int nrhs, bool load,
                  TuneEntry *out) {
    if (getenv("COLA_HOP_SHAPE") || h->flic) return false;
    TuneStore &ts = tune_store();
    std::lock_guard<std::mutex> lock(ts.mu);
    if (!ts.loaded && load) {
        ts.loaded = true;
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            std::map<std::string, TuneEntry> t;
            if (read_table(path, t) > 0)
                for (auto &kv : t) ts.table.emplace(kv.first, kv.second);  // keep newer
        }
    }
    auto it = ts.table.find(store_key(h, key));
    if (it == ts.table.end()) return false;
    TuneEntry e = it->second;
    if (!shape_valid(h->g, prec, nrhs, e)) return false;
    if (e.stage && !stage_ok(h->g, prec, nrhs, e)) e.stage = 0;
    *out = e;
    return true;
}

int tune_hop(cola_handle_t *h, const HopCall &c, int prec, int nrhs, TuneEntry *best,
             hipStream_t st) {
    std::vector<TuneEntry> cand;
    for (int rpt : {1, 2, 3, 4}) {
        if (nrhs % rpt) continue;
        if (rpt > 1 && spinor_fmt(prec) == SpinorFmt::F64) continue;
        const int G = nrhs / rpt;
        // blocks of whole wavefronts when some block size allows it
        bool whole = false;
        for (int T : {4, 8, 16, 32, 64, 128, 256}) whole |= T * G <= 256 && (T * G) % 64 == 0;
        for (int T : {4, 8, 16, 32, 64, 128, 256}) {
            if (T * G > 256 || T * G < 64) continue;
            if (whole && (T * G) % 64 != 0) continue;
            for (int tc : {1, 2, 4, 8, 16}) {
                if (h->g.L[3] % tc) continue;
                for (int grid : {0, -1}) {
                    TuneEntry t;
                    t.rpt = rpt;
                    t.sites_per_block = T;
                    t.grid = grid;
                    t.tchunk = tc;
                    cand.push_back(t);
                }
            }
            const int tiles[][2] = {{4, 4}, {8, 4}, {4, 8}, {8, 8}, {16, 8}, {8, 16}, {16, 16}};
            for (const auto &tl : tiles) {
                if (!tile_ok(h->g, tl[0], tl[1])) continue;
                TuneEntry t;
                t.rpt = rpt;
                t.sites_per_block = T;
                t.tile_y = tl[0];
                t.tile_z = tl[1];
                cand.push_back(t);
            }
        }
    }
    // each shape also with the site's links staged in LDS, where that applies
    const size_t n0 = cand.size();
    for (size_t k = 0; k < n0; ++k) {
        if (!stage_ok(h->g, prec, nrhs, cand[k])) continue;
        TuneEntry t = cand[k];
        t.stage = 1;
        cand.push_back(t);
        // the time walk of staged FP32 / FP16 hops: tiles in chunks of 4 and 8 timeslices
        if ((prec == COLA_FP32 || prec == COLA_FP16) && t.rpt == 1 && t.tile_y > 0) {
            for (int tc : {4, 8}) {
                if (h->g.L[3] % tc) continue;
                TuneEntry w = t;
                w.tchunk = tc;
                cand.push_back(w);
            }
        }
    }
    hipEvent_t e0, e1;
    COLA_HIP(h, hipEventCreate(&e0));
    COLA_HIP(h, hipEventCreate(&e1));
    double best_ms = 1e30;
    for (auto &t : cand) {
        COLA_TRY(fill_and_launch(h, c, prec, nrhs, t, st));  // warm-up
        COLA_HIP(h, hipEventRecord(e0, st));
        const int reps = 3;
        for (int k = 0; k < reps; ++k) COLA_TRY(fill_and_launch(h, c, prec, nrhs, t, st));
        COLA_HIP(h, hipEventRecord(e1, st));
        COLA_HIP(h, hipEventSynchronize(e1));
        float ms = 0;
        COLA_HIP(h, hipEventElapsedTime(&ms, e0, e1));
        t.ms = ms / reps;
        if (t.ms < best_ms) {
            best_ms = t.ms;
            *best = t;
        }
    }
    COLA_HIP(h, hipEventDestroy(e0));
    COLA_HIP(h, hipEventDestroy(e1));
    return COLA_OK;
}

}  // namespace

int flush_timing(cola_handle_t *h, bool wait_all) {
    size_t done = 0;
    for (; done < h->pending.size(); ++done) {
        auto &pr = h->pending[done];
        if (wait_all) {
            COLA_HIP(h, hipEventSynchronize(pr.second));
        } else if (hipEventQuery(pr.second) != hipSuccess) {
            break;
        }
        float ms = 0;
        COLA_HIP(h, hipEventElapsedTime(&ms, pr.first, pr.second));
        const int pi = h->pending_prec[done];
        const int ek = h->pending_epi[done];
        h->stats.hop_launches[pi] += 1;
        h->stats.hop_seconds[pi] += ms * 1e-3;
        h->stats.hop_bytes[pi] += h->pending_bytes[done];
        h->stats.hop_flops[pi] += h->pending_flops[done];
        h->stats.kind_launches[pi][ek] += 1;
        h->stats.kind_seconds[pi][ek] += ms * 1e-3;
        h->stats.kind_bytes[pi][ek] += h->pending_bytes[done];
        h->event_pool.push_back(pr.first);
        h->event_pool.push_back(pr.second);
    }
    h->pending.erase(h->pending.begin(), h->pending.begin() + done);
    h->pending_bytes.erase(h->pending_bytes.begin(), h->pending_bytes.begin() + done);
    h->pending_flops.erase(h->pending_flops.begin(), h->pending_flops.begin() + done);
    h->pending_prec.erase(h->pending_prec.begin(), h->pending_prec.begin() + done);
    h->pending_epi.erase(h->pending_epi.begin(), h->pending_epi.begin() + done);
    return COLA_OK;
}

int hop(cola_handle_t *h, const HopCall &c, int prec, int nrhs, hipStream_t st) {
    if (!h->gauge_set) return set_error(h, COLA_ESTATE, "no gauge field set");
    if (prec != COLA_FP64 && !h->su3)
        return set_error(h, COLA_EINVAL,
                         "compressed link formats need an SU(3) gauge field (check failed)");
    if (!h->gauge[(int)link_fmt(prec)])
        return set_error(h, COLA_EINVAL, "packed gauge field missing for this precision");
    if (h->flic && prec == COLA_FP16)
        return set_error(h, COLA_EINVAL, "the FLIC operator runs in FP64 and FP32");
    // The CG epilogues update their vectors in place, so they are never timed by the
    // tuner: they take the shape tuned for the epilogue they extend, else the default.
    const bool cg = c.epi == EPI_XPAY_CG || c.epi == EPI_CLOV_XPAY_CG;
    const int key_epi = c.epi == EPI_XPAY_CG ? EPI_XPAY
                        : c.epi == EPI_CLOV_XPAY_CG ? EPI_CLOV_XPAY
                                                    : c.epi;
    const std::string key = tune_key(h, prec, nrhs, key_epi, c.norm_result != nullptr);
    TuneEntry te;
    auto it = h->tune.find(key);
    if (it != h->tune.end() && (h->tune_mode != 2 || cg || c.fixed)) {
        te = it->second;
    } else if (h->tune_mode >= 1 && !cg && !c.fixed && !h->flic) {
        COLA_TRY(tune_hop(h, c, prec, nrhs, &te, st));
        h->tune[key] = te;
        // into the process-wide table and its file (a failed write only loses the cache)
        TuneStore &ts = tune_store();
        std::lock_guard<std::mutex> lock(ts.mu);
        ts.table[store_key(h, key)] = te;
        const std::string path = tune_cache_path();
        if (!path.empty()) write_table(path, ts.table);
    } else if (!stored_entry(h, key, prec, nrhs, !c.fixed, &te)) {
        te = default_entry(h->g, prec, nrhs);
    }
    // a resident grid needs an occupancy query (cached in a host map): the fixed mode
    // takes the plain grid instead, which gives bitwise the same output
    if (c.fixed && te.grid < 0) te.grid = 0;
    // FLIC hops: one rhs per lane, both links loaded per lane
    if (h->flic) {
        te.rpt = 1;
        te.stage = 0;
    }
    const bool timed = (h->flags & COLA_FLAG_TIMING) != 0 && !c.fixed;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        if (h->pending.size() > 2048) COLA_TRY(flush_timing(h, false));
        if (h->pending.size() > 4096) COLA_TRY(flush_timing(h, true));
        e0 = take_event(h);
        e1 = take_event(h);
        if (!e0 || !e1) return set_error(h, COLA_EHIP, "hipEventCreate failed");
        COLA_HIP(h, hipEventRecord(e0, st));
    }
    int grid = 0;
    COLA_TRY(fill_and_launch(h, c, prec, nrhs, te, st, false, &grid));
    if (timed) COLA_HIP(h, hipEventRecord(e1, st));
    if (c.norm_result)
        COLA_HIP(h, launch_reduce_partials(h->partial, grid, nrhs, c.norm_result, st));
    if (timed) {
        double b, f;
        hop_work(h, prec, nrhs, c.epi, &b, &f);
        h->pending.push_back({e0, e1});
        h->pending_bytes.push_back(b);
        h->pending_flops.push_back(f);
        h->pending_prec.push_back(prec);
        h->pending_epi.push_back(c.epi);
    }
    return COLA_OK;
}

int tune_cache_load(cola_handle_t *h, const char *path) {
    const std::string p = path ? path : tune_cache_path();
    if (p.empty()) return set_error(h, COLA_EINVAL, "no tuning cache path");
    std::map<std::string, TuneEntry> t;
    const int n = read_table(p, t);
    if (n < 0) return set_error(h, COLA_EINVAL, "cannot read " + p);
    TuneStore &ts = tune_store();
    std::lock_guard<std::mutex> lock(ts.mu);
    ts.loaded = true;
    for (auto &kv : t) ts.table[kv.first] = kv.second;
    return n;
}

int tune_cache_save(cola_handle_t *h, const char *path) {
    const std::string p = path ? path : tune_cache_path();
    if (p.empty()) return set_error(h, COLA_EINVAL, "no tuning cache path");
    TuneStore &ts = tune_store();
    std::lock_guard<std::mutex> lock(ts.mu);
    const int n = write_table(p, ts.table);
    if (n < 0) return set_error(h, COLA_EINVAL, "cannot write " + p);
    return n;
}

size_t op_workspace_bytes(const cola_handle_t *h, int op, int prec, int nrhs) {
    const size_t bb = spinor_block_bytes(h->g, spinor_fmt(prec), nrhs);
    switch (op) {
        case COLA_OP_SCHUR:
        case COLA_OP_SCHUR_DAG: return bb;
        case COLA_OP_SCHUR_DAGSCHUR:
        case COLA_OP_MDAGM: return 2 * bb;
        default: return 0;
    }
}

int apply_op(cola_handle_t *h, void *out, const void *in, int op, int parity, int prec, int nrhs,
             hipStream_t st, double *norm_result, char *ws) {
    const SpinorFmt sf = spinor_fmt(prec);
    const size_t bb = spinor_block_bytes(h->g, sf, nrhs);
    const bool fixed = ws != nullptr;
    const bool clover = h->csw != 0.0;
    const bool f64 = sf == SpinorFmt::F64;
    const void *A = f64 ? h->clov64 : h->clov32;
    const void *Ainv = f64 ? h->clovinv64 : h->clovinv32;
    const double k = h->kappa;
    auto blk = [bb](const void *base, int p) { return (void *)((const char *)base + p * bb); };

    switch (op) {
        case COLA_OP_HOP:
        case COLA_OP_HOP_DAG: {
            HopCall c{out, in, parity, op == COLA_OP_HOP_DAG ? 1 : 0};
            c.norm_result = norm_result;
            c.fixed = fixed;
            return hop(h, c, prec, nrhs, st);
        }
        case COLA_OP_M:
        case COLA_OP_MDAG: {
            // out_p = A_pp in_p - kappa D_{p,1-p} in_{1-p}
            const int dag = op == COLA_OP_MDAG;
            for (int p = 0; p < 2; ++p) {
                HopCall c{blk(out, p), blk(in, 1 - p), p, dag};
                c.epi = clover ? EPI_CLOV_XPAY : EPI_XPAY;
                c.x = blk(in, p);
                c.a = -k;
                c.clov = A;
                c.fixed = fixed;
                COLA_TRY(hop(h, c, prec, nrhs, st));
            }
            return COLA_OK;
        }
        case COLA_OP_MDAGM: {
            void *t = ws;
            if (!fixed)
                COLA_TRY(get_vec(h, "op_full_" + std::to_string((int)sf) + "_" +
                                        std::to_string(nrhs), 2 * bb, &t));
            COLA_TRY(apply_op(h, t, in, COLA_OP_M, -1, prec, nrhs, st, nullptr, ws));
            return apply_op(h, out, t, COLA_OP_MDAG, -1, prec, nrhs, st, nullptr, ws);
        }
        case COLA_OP_SCHUR:
        case COLA_OP_SCHUR_DAG: {
            // t_o = A_oo^-1 D_oe in_e ; out_e = A_ee in_e - kappa^2 D_eo t_o
            const int dag = op == COLA_OP_SCHUR_DAG;
            void *t = ws;
            if (!fixed)
                COLA_TRY(get_vec(h, "op_odd_" + std::to_string((int)sf) + "_" +
                                        std::to_string(nrhs), bb, &t));
            HopCall c1{t, in, 1, dag};
            if (clover) {
                c1.epi = EPI_CLOV;
                c1.clov = Ainv;
            }
            c1.fixed = fixed;
            COLA_TRY(hop(h, c1, prec, nrhs, st));
            HopCall c2{out, t, 0, dag};
            c2.epi = clover ? EPI_CLOV_XPAY : EPI_XPAY;
            c2.x = in;
            c2.a = -k * k;
            c2.clov = A;
            c2.norm_result = norm_result;
            c2.fixed = fixed;
            return hop(h, c2, prec, nrhs, st);
        }
        case COLA_OP_SCHUR_DAGSCHUR: {
            // fixed workspace: [even t | odd intermediate of each Schur factor]
            void *t = ws;
            if (!fixed)
                COLA_TRY(get_vec(h, "op_even_" + std::to_string((int)sf) + "_" +
                                        std::to_string(nrhs), bb, &t));
            char *ws2 = fixed ? ws + bb : nullptr;
            COLA_TRY(apply_op(h, t, in, COLA_OP_SCHUR, 0, prec, nrhs, st, norm_result, ws2));
            return apply_op(h, out, t, COLA_OP_SCHUR_DAG, 0, prec, nrhs, st, nullptr, ws2);
        }
        default: return set_error(h, COLA_EINVAL, "unknown operator");
    }
}

int schur_normal_cg_step(cola_handle_t *h, int prec, int nrhs, hipStream_t st, void *x, void *r,
                         const void *p, const double *rho, double *pi, const int *active,
                         double *rho_new) {
    const SpinorFmt sf = spinor_fmt(prec);
    const size_t bb = spinor_block_bytes(h->g, sf, nrhs);
    const bool clover = h->csw != 0.0;
    const bool f64 = sf == SpinorFmt::F64;
    void *te, *to;
    // the same work vectors as COLA_OP_SCHUR_DAGSCHUR and COLA_OP_SCHUR
    COLA_TRY(get_vec(h, "op_even_" + std::to_string((int)sf) + "_" + std::to_string(nrhs), bb,
                     &te));
    COLA_TRY(get_vec(h, "op_odd_" + std::to_string((int)sf) + "_" + std::to_string(nrhs), bb,
                     &to));
    COLA_TRY(apply_op(h, te, p, COLA_OP_SCHUR, 0, prec, nrhs, st, pi));
    // S^dag te: t_o = A_oo^-1 D_oe^dag te, then the CG update with A_ee te - kappa^2 D_eo^dag t_o
    HopCall c1{to, te, 1, 1};
    if (clover) {
        c1.epi = EPI_CLOV;
        c1.clov = f64 ? h->clovinv64 : h->clovinv32;
    }
    COLA_TRY(hop(h, c1, prec, nrhs, st));
    HopCall c2{r, to, 0, 1};
    c2.epi = clover ? EPI_CLOV_XPAY_CG : EPI_XPAY_CG;
    c2.x = te;
    c2.a = -h->kappa * h->kappa;
    c2.clov = f64 ? h->clov64 : h->clov32;
    c2.norm_result = rho_new;
    c2.cg_x = x;
    c2.cg_r = r;
    c2.cg_p = p;
    c2.cg_rho = rho;
    c2.cg_pi = pi;
    c2.cg_active = active;
    return hop(h, c2, prec, nrhs, st);
}

}  // namespace cola
