// C ABI of the PMMM far-field library: plan objects, parameter checks,
// workspace management and the launch sequence of one far-field call.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pmmm_hier.h"

namespace pmmm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

hipError_t set_max_lds(const void *kernel, size_t bytes) {
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(kernel);
    if (it != done.end() && it->second >= bytes) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done[kernel] = bytes;
    return e;
}

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? PMMM_ENOMEM : PMMM_EHIP;
}

// P2M: a cell of more than 16 G particles (G lanes per light cell, so at
// most 16 particles per lane there) is cut into dense items of kDenseItem
// particles, one wave each.
static int dense_threshold_for(int group) { return 16 * group; }

// From this many particles on, L2P writes its results in sorted order and a
// second kernel sends them back to the caller's order (fewer, wider random
// accesses); below it the extra launch costs more than it saves.
constexpr int64_t kStagedL2PMinN = int64_t(1) << 18;

struct Plan {
    pmmm_params prm;
    int n, nf, p, P, Q, open, prec, cutoff, images;
    int lim[3];               // cells per axis of the caller's box (open: a corner of n^3)
    int generic;              // periodic n not a power of two: direct-DFT stages
    void *spec2 = nullptr;    // generic: M2L output spectra
    // fine plan of a hierarchy: no transfer kernel or spectra; its far
    // stage is the local M2L over hier_table (margin hier_D, refinement hier_r)
    bool no_transfer = false;
    const float *hier_table = nullptr;
    int hier_r = 0, hier_D = 0;
    int64_t K, ncol, ngreen;  // ngreen: stored transfer-kernel values
    double box, h, inv_h, alpha, alpha_cell;
    int device;
    size_t tsize;
    // plan-lifetime buffers
    void *green = nullptr, *tw = nullptr, *M = nullptr, *spec = nullptr, *L = nullptr;
    int *start = nullptr, *small = nullptr;
    int *tile_first = nullptr;  // near field: first tile of every row of cells
    double *sums = nullptr, *qr2_partial = nullptr;
    // particle buffers
    int64_t cap = 0, last_n = -1;
    int *cell_of = nullptr, *slot = nullptr, *perm = nullptr, *scell = nullptr, *pos = nullptr;
    int *tile_row = nullptr;    // near field: row of every tile
    int *count = nullptr, *tile_sums = nullptr;  // radix-sort histograms and scan scratch
    void *sorted = nullptr, *staged = nullptr;   // staged: out4<T>[cap] sorted-order results
    int4 *items = nullptr;                       // dense P2M items [dense_items_cap(cap, K)]
    float *partial = nullptr;                    // [dense_slots_cap(cap)][P + 1]
    hipStream_t last_stream = nullptr;
    // multi-charge workspace (chunks of up to kMultiMaxSets sets)
    int mcap_sets = 0;
    float *mM = nullptr;          // [K][P+1][S] moments, then [K][P][S] local expansions
    void *mY = nullptr;           // [nf][nf][nf/2+1][P S] spectra
    unsigned *mtmap = nullptr;    // t-matrix map in MFMA fragment order
    double *mqr2 = nullptr, *mqtot = nullptr;
    // tuned launch shapes (0: defaults)
    int tune_col_w = 0, tune_group = 0, tune_col_kernel = 0;
    // graph replay of repeated calls (pmmm_plan_set_graphs)
    int use_graph = 0;
    std::vector<intptr_t> gkey;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // stage timing
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[PMMM_NSTAGES];
    double prof_ms[PMMM_NSTAGES] = {0};
    int64_t prof_cnt[PMMM_NSTAGES] = {0};
};

// Brackets one stage of a far-field call with HIP events when profiling is on.
struct StageTimer {
    Plan *pl;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(Plan *pl_, int st, hipStream_t s_, bool enabled = true)
        : pl(pl_), stage(st), s(s_) {
        if (!enabled || !(pl->prof_mask & (1u << stage))) return;
        a = take();
        b = take();
        if (a) hipEventRecord(a, s);
    }
    hipEvent_t take() {
        if (!pl->ev_pool.empty()) {
            hipEvent_t e = pl->ev_pool.back();
            pl->ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~StageTimer() {
        if (!a || !b) return;
        hipEventRecord(b, s);
        pl->ev_pending[stage].push_back({a, b});
    }
};

}  // namespace pmmm

struct pmmm_plan_s : pmmm::Plan {};

using namespace pmmm;

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Cells per axis of the mesh the library computes on.  A periodic mesh is
// the caller's (cubic, power of two).  An open mesh of nx x ny x nz cubic
// cells is computed on the smallest power-of-two cube of the same cells
// that holds it (at least 4 per axis): the open convolution is linear, so
// the extra cells, which hold no particles, change no result, and the near
// cube of every cell is the same.
static int mesh_cells(const pmmm_params *prm) {
    if (prm->boundary != PMMM_OPEN) return prm->nx;
    int n = 4;
    while (n < prm->nx || n < prm->ny || n < prm->nz) n *= 2;
    return n;
}

static int validate(const pmmm_params *prm, std::string &why) {
    if (!prm) {
        why = "params is NULL";
        return PMMM_EINVAL;
    }
    if (prm->nx < 1 || prm->ny < 1 || prm->nz < 1) {
        why = "mesh dimensions must be positive";
        return PMMM_EINVAL;
    }
    if (!(prm->box[0] > 0 && prm->box[1] > 0 && prm->box[2] > 0)) {
        why = "box lengths must be positive";
        return PMMM_EINVAL;
    }
    const double h0 = prm->box[0] / prm->nx, h1 = prm->box[1] / prm->ny, h2 = prm->box[2] / prm->nz;
    if (std::fabs(h0 - h1) > 1e-12 * h0 || std::fabs(h0 - h2) > 1e-12 * h0) {
        why = "cells must be cubic (box[a]/n[a] equal)";
        return PMMM_EINVAL;
    }
    if (prm->p < 0 || prm->p > PMMM_PMAX) {
        why = "p outside 0..PMMM_PMAX";
        return PMMM_EINVAL;
    }
    const int c = prm->cutoff == 0 ? 2 : prm->cutoff;
    if (c != 1 && c != 2) {
        why = "cutoff must be 1 or 2";
        return PMMM_EINVAL;
    }
    if (prm->boundary != PMMM_OPEN && prm->boundary != PMMM_PERIODIC) {
        why = "boundary must be PMMM_OPEN or PMMM_PERIODIC";
        return PMMM_EINVAL;
    }
    if (prm->precision != PMMM_F32 && prm->precision != PMMM_F64 &&
        prm->precision != PMMM_BF16X3) {
        why = "precision must be PMMM_F32, PMMM_F64 or PMMM_BF16X3";
        return PMMM_EINVAL;
    }
    if (prm->alpha < 0 || prm->images < 0 || prm->n_max < 0) {
        why = "alpha, images and n_max must be non-negative";
        return PMMM_EINVAL;
    }
    const int n = mesh_cells(prm);
    if (prm->boundary == PMMM_PERIODIC && n < 2 * c + 1) {
        why = "periodic mesh needs n >= 2c + 1";
        return PMMM_EINVAL;
    }
    if (prm->boundary == PMMM_PERIODIC && (prm->nx != prm->ny || prm->nx != prm->nz)) {
        why = "periodic meshes must be cubic";
        return PMMM_EUNSUPPORTED;
    }
    if (prm->boundary == PMMM_PERIODIC && !is_pow2(n) && n > kGenericMaxN) {
        why = "periodic meshes whose edge is not a power of two are limited to 64 cells per axis";
        return PMMM_EUNSUPPORTED;
    }
    const int nf = prm->boundary == PMMM_OPEN ? 2 * n : n;
    const int nfmax = prm->precision == PMMM_F64 ? 64 : 128;
    if (nf > nfmax) {
        why = "FFT mesh too large for the library (FP32: nf <= 128, FP64: nf <= 64)";
        return PMMM_EUNSUPPORTED;
    }
    // the column kernel keeps at least one column's spectra in LDS (160 KB per CU)
    if (is_pow2(n) && column_default_kernel(prm->p, nf, prm->precision == PMMM_F64 ? 8 : 4) == 0) {
        why = "order too high for this FFT mesh: one column's spectra exceed 160 KB of LDS";
        return PMMM_EUNSUPPORTED;
    }
    return PMMM_OK;
}

static void derive(Plan *pl, const pmmm_params *prm) {
    pl->prm = *prm;
    pl->n = mesh_cells(prm);
    pl->lim[0] = prm->nx;
    pl->lim[1] = prm->ny;
    pl->lim[2] = prm->nz;
    pl->generic = !is_pow2(pl->n);
    pl->open = prm->boundary == PMMM_OPEN;
    pl->nf = pl->open ? 2 * pl->n : pl->n;
    pl->p = prm->p;
    pl->P = nreal(pl->p);
    pl->Q = nreal(2 * pl->p);
    pl->prec = prm->precision;
    pl->cutoff = prm->cutoff == 0 ? 2 : prm->cutoff;
    pl->images = prm->images == 0 ? 4 : prm->images;
    pl->K = (int64_t)pl->n * pl->n * pl->n;
    pl->ncol = (int64_t)pl->nf * (pl->nf / 2 + 1);
    {
        const int64_t nh = pl->nf / 2 + 1, nhp = (nh + 3) & ~3;
        pl->ngreen = nh * nh * pl->Q * nhp;
    }
    // box: edge of the computed cube (the caller's, or its embedding)
    pl->box = pl->n == prm->nx ? prm->box[0] : prm->box[0] / prm->nx * pl->n;
    pl->h = pl->box / pl->n;
    pl->inv_h = pl->n / pl->box;
    pl->alpha = prm->alpha == 0 ? 1.5 / pl->box : prm->alpha;
    pl->alpha_cell = pl->alpha * pl->h;
    pl->tsize = pl->prec == PMMM_F64 ? 8 : 4;
}

static size_t plan_bytes(const Plan *pl) {
    const size_t t = pl->tsize, c = 2 * t;
    size_t b = 0;
    b += (size_t)pl->ngreen * t;                         // green
    b += (size_t)(pl->generic ? pl->nf : pl->nf / 2) * c; // twiddles
    if (pl->generic) b += (size_t)pl->P * pl->n * pl->ncol * c;  // M2L output spectra
    b += (size_t)(pl->P + 1) * pl->K * t;                // M
    b += (size_t)pl->P * pl->n * pl->ncol * c;           // spectra
    b += (size_t)pl->P * pl->K * t;                      // L
    b += ((size_t)pl->K + 1 + 8) * sizeof(int);                                   // starts, small
    b += 8 * sizeof(double) + (size_t)pl->n * sizeof(double);                     // sums, plane sums
    b += (size_t)pl->n * pl->n * sizeof(int);                                     // near-field row tiles
    return b;
}

static size_t particle_bytes(const Plan *pl, int64_t n) {
    return (size_t)n * (5 * sizeof(int) + 8 * pl->tsize) +
           sizeof(int) * (size_t)(near_tile_capacity(n, pl->n) + bin_hist_ints(n) +
                                  bin_scan_tiles(n)) +
           sizeof(int4) * (size_t)dense_items_cap(n, pl->K) +
           sizeof(float) * (size_t)dense_slots_cap(n) * (pl->P + 1);
}

static void free_particles(Plan *pl) {
    hipFree(pl->cell_of);
    hipFree(pl->slot);
    hipFree(pl->perm);
    hipFree(pl->scell);
    hipFree(pl->sorted);
    hipFree(pl->pos);
    hipFree(pl->staged);
    hipFree(pl->tile_row);
    hipFree(pl->count);
    hipFree(pl->tile_sums);
    hipFree(pl->items);
    hipFree(pl->partial);
    pl->cell_of = pl->slot = pl->perm = pl->scell = pl->pos = pl->tile_row = nullptr;
    pl->count = pl->tile_sums = nullptr;
    pl->sorted = pl->staged = nullptr;
    pl->items = nullptr;
    pl->partial = nullptr;
    pl->cap = 0;
}

static int ensure_capacity(Plan *pl, int64_t n) {
    if (n <= pl->cap) return PMMM_OK;
    if (n > (int64_t)INT32_MAX) {
        set_error("particle count exceeds the 32-bit index range");
        return PMMM_EINVAL;
    }
    PMMM_HIP(hipDeviceSynchronize());
    free_particles(pl);
    PMMM_HIP(hipMalloc(&pl->cell_of, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&pl->slot, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&pl->perm, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&pl->scell, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&pl->sorted, 4 * pl->tsize * n));
    PMMM_HIP(hipMalloc(&pl->pos, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&pl->staged, 4 * pl->tsize * n));
    PMMM_HIP(hipMalloc(&pl->tile_row, sizeof(int) * near_tile_capacity(n, pl->n)));
    PMMM_HIP(hipMalloc(&pl->count, sizeof(int) * bin_hist_ints(n)));
    PMMM_HIP(hipMalloc(&pl->tile_sums, sizeof(int) * bin_scan_tiles(n)));
    PMMM_HIP(hipMalloc(&pl->items, sizeof(int4) * dense_items_cap(n, pl->K)));
    PMMM_HIP(hipMalloc(&pl->partial, sizeof(float) * dense_slots_cap(n) * (pl->P + 1)));
    pl->cap = n;
    return PMMM_OK;
}

static void drop_plan_graph(Plan *pl) {
    if (pl->gexec) hipGraphExecDestroy(pl->gexec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    pl->gexec = nullptr;
    pl->graph = nullptr;
    pl->gkey.clear();
}

static void destroy(Plan *pl) {
    if (!pl) return;
    hipDeviceSynchronize();
    drop_plan_graph(pl);
    free_particles(pl);
    hipFree(pl->green);
    hipFree(pl->tw);
    hipFree(pl->M);
    hipFree(pl->spec);
    hipFree(pl->spec2);
    hipFree(pl->L);
    hipFree(pl->start);
    hipFree(pl->small);
    hipFree(pl->tile_first);
    hipFree(pl->sums);
    hipFree(pl->qr2_partial);
    hipFree(pl->mM);
    hipFree(pl->mY);
    hipFree(pl->mtmap);
    hipFree(pl->mqr2);
    hipFree(pl->mqtot);
    for (hipEvent_t e : pl->ev_pool) hipEventDestroy(e);
    for (auto &v : pl->ev_pending)
        for (auto &pr : v) {
            hipEventDestroy(pr.first);
            hipEventDestroy(pr.second);
        }
    delete static_cast<pmmm_plan_s *>(pl);
}

// Radix-2 twiddles e^(-2 pi i k / nf), k < nf/2; a generic plan keeps all nf
// roots of unity for its direct DFTs.
template <typename T>
static int make_twiddles(Plan *pl, hipStream_t s) {
    const int nf = pl->nf, cnt = pl->generic ? nf : nf / 2;
    std::vector<cplx<T>> tw(cnt);
    for (int k = 0; k < cnt; ++k)
        tw[k] = {T(std::cos(2.0 * M_PI * k / nf)), T(-std::sin(2.0 * M_PI * k / nf))};
    PMMM_HIP(hipMalloc(&pl->tw, sizeof(cplx<T>) * cnt));
    PMMM_HIP(hipMemcpyAsync(pl->tw, tw.data(), sizeof(cplx<T>) * cnt, hipMemcpyHostToDevice, s));
    return PMMM_OK;
}

static int alloc_plan(Plan *pl, hipStream_t s) {
    const size_t t = pl->tsize, c = 2 * t;
    if (!pl->no_transfer) {
        PMMM_HIP(hipMalloc(&pl->green, (size_t)pl->ngreen * t));
        PMMM_HIP(hipMalloc(&pl->spec, (size_t)pl->P * pl->n * pl->ncol * c));
        if (pl->generic) PMMM_HIP(hipMalloc(&pl->spec2, (size_t)pl->P * pl->n * pl->ncol * c));
    }
    PMMM_HIP(hipMalloc(&pl->M, (size_t)(pl->P + 1) * pl->K * t));
    PMMM_HIP(hipMalloc(&pl->L, (size_t)pl->P * pl->K * t));
    PMMM_HIP(hipMalloc(&pl->start, sizeof(int) * (pl->K + 1)));
    // [0] dense items, [1] domain flag, [2] near tiles, [3] partial slots
    PMMM_HIP(hipMalloc(&pl->small, sizeof(int) * 8));
    PMMM_HIP(hipMalloc(&pl->tile_first, sizeof(int) * (size_t)pl->n * pl->n));
    PMMM_HIP(hipMalloc(&pl->sums, sizeof(double) * 8));
    PMMM_HIP(hipMalloc(&pl->qr2_partial, sizeof(double) * pl->n));
    PMMM_HIP(hipMemsetAsync(pl->small, 0, sizeof(int) * 8, s));
    PMMM_HIP(hipMemsetAsync(pl->sums, 0, sizeof(double) * 8, s));
    PMMM_HIP(hipMemsetAsync(pl->M, 0, (size_t)(pl->P + 1) * pl->K * t, s));
    return pl->prec == PMMM_F64 ? make_twiddles<double>(pl, s) : make_twiddles<float>(pl, s);
}

// Lanes per cell in the light P2M path: about four particles per lane.
static int group_for(double mean) {
    if (mean <= 24) return 4;
    if (mean <= 48) return 8;
    if (mean <= 96) return 16;
    if (mean <= 192) return 32;
    return 64;
}

// What one call computes: the far field (pmmm_far_*), the near field alone
// (pmmm_near_*) or both with one binning (pmmm_total_*).
// kHierFine / kHierTotal: the fine level of a hierarchy (and its near field),
// added into outputs that already hold the coarse far field
enum CallMode { kFar = 0, kNear = 1, kTotal = 2, kHierFine = 3, kHierTotal = 4 };

// Per-particle device buffers of one call: the plan's own (grown on demand)
// or, for the allocation-free entry point, slices of the static scratch.
struct PBuf {
    int *cell_of, *slot, *perm, *scell, *pos, *tile_row, *count, *tile_sums;
    void *sorted, *staged;
    int4 *items;
    float *partial;
    int64_t items_cap, slots_cap;
};

static PBuf plan_pbuf(const Plan *pl) {
    return PBuf{pl->cell_of,    pl->slot,   pl->perm,   pl->scell,
                pl->pos,        pl->tile_row, pl->count, pl->tile_sums,
                pl->sorted,     pl->staged, pl->items,  pl->partial,
                dense_items_cap(pl->cap, pl->K), dense_slots_cap(pl->cap)};
}

// ext == nullptr: the plan's particle buffers, grown to n if needed (which
// allocates) and stage timing as configured; otherwise the caller's buffers
// (capacity checked by the caller), no allocation and no events.
template <typename T>
static int enqueue_impl(pmmm_plan_s *pl, CallMode mode, int64_t n, const T *x, const T *y,
                        const T *z, const T *q, T *phi, T *gx, T *gy, T *gz, int accumulate,
                        const PBuf &pb, bool timed, hipStream_t s);

template <typename T>
static int call_impl(pmmm_plan_s *pl, CallMode mode, int64_t n, const T *x, const T *y,
                     const T *z, const T *q, T *phi, T *gx, T *gy, T *gz, int accumulate,
                     void *stream, const PBuf *ext = nullptr) {
    if (!pl) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    if (sizeof(T) != pl->tsize) {
        set_error("precision of the call does not match the plan");
        return PMMM_EINVAL;
    }
    if (n < 0) {
        set_error("n must be non-negative");
        return PMMM_EINVAL;
    }
    if (n > 0 && (!x || !y || !z || !q || !phi || !gx || !gy || !gz)) {
        set_error("NULL particle or output pointer");
        return PMMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    PMMM_HIP(hipGetDevice(&cur));
    if (cur != pl->device) {
        set_error("current device differs from the plan's device");
        return PMMM_EINVAL;
    }
    if (ext == nullptr) {
        const int rc = ensure_capacity(pl, n > 0 ? n : 1);
        if (rc != PMMM_OK) return rc;
    }
    const PBuf pb = ext != nullptr ? *ext : plan_pbuf(pl);
    const bool timed = ext == nullptr;
    pl->last_stream = s;
    pl->last_n = n;
    if (pl->use_graph && ext == nullptr && pl->prof_mask == 0 && s != nullptr) {
        // a call repeating the previous one (same mode, sizes, pointers,
        // stream and launch shapes) replays it as a graph: the second such
        // call captures the launches, later ones only launch the graph
        const std::vector<intptr_t> key = {
            (intptr_t)mode, (intptr_t)n, (intptr_t)x, (intptr_t)y, (intptr_t)z, (intptr_t)q,
            (intptr_t)phi, (intptr_t)gx, (intptr_t)gy, (intptr_t)gz, (intptr_t)accumulate,
            (intptr_t)s, (intptr_t)pb.cell_of, (intptr_t)pb.staged, (intptr_t)pb.items,
            (intptr_t)pl->tune_group, (intptr_t)pl->tune_col_kernel, (intptr_t)pl->tune_col_w};
        if (key == pl->gkey) {
            if (pl->gexec == nullptr) {
                PMMM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                const int rc = enqueue_impl<T>(pl, mode, n, x, y, z, q, phi, gx, gy, gz,
                                               accumulate, pb, false, s);
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(s, &g);
                if (rc != PMMM_OK) {
                    if (g) hipGraphDestroy(g);
                    return rc;
                }
                PMMM_HIP(e);
                pl->graph = g;
                PMMM_HIP(hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0));
            }
            PMMM_HIP(hipGraphLaunch(pl->gexec, s));
            return PMMM_OK;
        }
        drop_plan_graph(pl);
        pl->gkey = key;
    }
    return enqueue_impl<T>(pl, mode, n, x, y, z, q, phi, gx, gy, gz, accumulate, pb, timed, s);
}

// The launches of one call, after its arguments have been checked.
template <typename T>
static int enqueue_impl(pmmm_plan_s *pl, CallMode mode, int64_t n, const T *x, const T *y,
                        const T *z, const T *q, T *phi, T *gx, T *gy, T *gz, int accumulate,
                        const PBuf &pb, bool timed, hipStream_t s) {
    // near and total calls, and large far-field calls, stage their results
    // as 16-byte records and send them to the outputs in one pass: in
    // sorted order (with each particle's sorted slot from the binning) when
    // the near field adds to them, else at the caller's indices
    const bool staged = mode != kFar || n >= kStagedL2PMinN;
    const bool sorted_stage = mode == kNear || mode == kTotal || mode == kHierTotal;
    const int group = pl->tune_group > 0 ? pl->tune_group : group_for((double)n / (double)pl->K);
    const int dense_thr = dense_threshold_for(group);

    {
        StageTimer t(pl, PMMM_STAGE_BIN, s, timed);
        BinArgs b{};
        b.n = n;
        b.x = x;
        b.y = y;
        b.z = z;
        b.q = q;
        b.ncell = pl->n;
        b.inv_h = pl->inv_h;
        b.periodic = !pl->open;
        for (int a3 = 0; a3 < 3; ++a3) b.lim[a3] = pl->lim[a3];
        b.cell_of = pb.cell_of;
        b.slot = pb.slot;
        b.count = pb.count;
        b.start = pl->start;
        b.scell = pb.scell;
        b.perm = pb.perm;
        b.flag = pl->small + 1;
        b.items = mode != kNear ? pb.items : nullptr;
        b.items_cap = pb.items_cap;
        b.slots_cap = pb.slots_cap;
        b.small = pl->small;
        b.pos = sorted_stage ? pb.pos : nullptr;
        b.tile_sums = pb.tile_sums;
        b.dense_threshold = dense_thr;
        b.sorted = pb.sorted;
        b.recs = pb.staged;   // free until L2P
        PMMM_HIP(launch_bin<T>(b, s));
    }
    if (mode != kNear) {
        {
            StageTimer t(pl, PMMM_STAGE_P2M, s, timed);
            P2MArgs m{};
            m.p = pl->p;
            m.ncell = pl->n;
            m.group = group;
            m.start = pl->start;
            m.dense_threshold = dense_thr;
            m.items = pb.items;
            m.items_cap = pb.items_cap;
            m.small = pl->small;
            m.partial = pb.partial;
            m.slots_cap = pb.slots_cap;
            m.sorted = pb.sorted;
            m.M = pl->M;
            PMMM_HIP(launch_p2m<T>(m, s));
        }
        FFTArgs f{};
        f.p = pl->p;
        f.n = pl->n;
        f.nf = pl->nf;
        f.open = pl->open;
        f.M = pl->M;
        f.spec = pl->spec;
        f.green = pl->green;
        f.tw = pl->tw;
        f.L = pl->L;
        f.qr2_partial = pl->qr2_partial;
        f.sums = pl->sums;
        f.col_w = pl->tune_col_w;
        f.col_kernel = pl->tune_col_kernel;
        f.generic = pl->generic;
        f.spec2 = pl->spec2;
        if (mode == kHierFine || mode == kHierTotal) {
            StageTimer t(pl, PMMM_STAGE_COLUMN, s, timed);
            HierArgs h{};
            h.p = pl->p;
            h.nf = pl->n;
            h.r = pl->hier_r;
            h.cutoff = pl->cutoff;
            h.D = pl->hier_D;
            h.M = (const float *)pl->M;
            h.L = (float *)pl->L;
            h.table = pl->hier_table;
            PMMM_HIP(launch_hier_m2l_f32(h, s));
        } else {
            for (int st = 0; st < 3; ++st) {
                StageTimer t(pl, PMMM_STAGE_FFT_FWD + st, s, timed);
                PMMM_HIP(launch_conv_stage<T>(f, st, s));
            }
        }
        {
            StageTimer t(pl, PMMM_STAGE_L2P, s, timed);
            L2PArgs l{};
            l.n = n;
            l.p = pl->p;
            l.ncell = pl->n;
            l.periodic = !pl->open;
            l.sorted = pb.sorted;
            l.scell = pb.scell;
            l.perm = pb.perm;
            l.L = pl->L;
            l.sums = pl->sums;
            l.alpha_cell = pl->alpha_cell;
            l.inv_h = pl->inv_h;
            l.phi = phi;
            l.gx = gx;
            l.gy = gy;
            l.gz = gz;
            if (staged) {
                l.staged = pb.staged;
                l.pos = sorted_stage ? pb.pos : nullptr;
            }
            PMMM_HIP(launch_l2p<T>(l, s));
            if (mode == kFar && staged)
                PMMM_HIP(launch_unpermute<T>(n, nullptr, pb.staged, phi, gx, gy, gz, 0, s));
            if (mode == kHierFine)   // added to the coarse far field already in the outputs
                PMMM_HIP(launch_unpermute<T>(n, nullptr, pb.staged, phi, gx, gy, gz, 1, s));
        }
    }
    if (mode == kNear || mode == kTotal || mode == kHierTotal) {
        StageTimer t(pl, PMMM_STAGE_NEAR, s, timed);
        NearArgs a{};
        a.n = n;
        a.ncell = pl->n;
        a.cutoff = pl->cutoff;
        a.periodic = !pl->open;
        a.accumulate = mode == kNear ? 0 : 1;
        a.start = pl->start;
        a.scell = pb.scell;
        a.sorted = pb.sorted;
        a.inv_h = pl->inv_h;
        a.tile_first = pl->tile_first;
        a.tile_row = pb.tile_row;
        a.ntiles = pl->small + 2;
        a.staged = pb.staged;
        PMMM_HIP(launch_near<T>(a, s));
        PMMM_HIP(launch_unpermute<T>(n, pb.pos, pb.staged, phi, gx, gy, gz,
                                     mode == kNear ? accumulate : (mode == kHierTotal ? 1 : 0), s));
    }
    return PMMM_OK;
}

// ------------------------------------------- allocation-free far field
// Per-particle scratch of pmmm_far_f32_noalloc in one file-scope device
// array: cell, slot, permutation, sorted cell and sorted-slot arrays (5 ints
// per particle), the sorted records and sorted-order results (two 16-byte
// records per particle), the radix-sort histograms, and the dense P2M items
// and partial sums (for orders up to PMMM_PMAX), each region 256-byte
// aligned.  Every region is written before it is read within a call (the
// item counts are reset by the binning), so nothing needs clearing.
constexpr int64_t kNoAllocMaxN = PMMM_NOALLOC_MAX_N;
constexpr size_t kNoAllocInts = (size_t)kNoAllocMaxN * sizeof(int);
constexpr size_t kNoAllocRecs = (size_t)kNoAllocMaxN * sizeof(particle4<float>);
// radix-sort histograms (512 buckets per tile) and their scan scratch
constexpr size_t kNoAllocHist = (size_t)bin_hist_ints(kNoAllocMaxN) * sizeof(int);
constexpr size_t kNoAllocSums = ((size_t)bin_scan_tiles(kNoAllocMaxN) * sizeof(int) + 255) / 256 * 256;
// dense items: at most max_n / (threshold + 1) dense cells whatever the mesh
constexpr int64_t kNoAllocItemsCap = dense_items_cap(kNoAllocMaxN, kNoAllocMaxN);
constexpr int64_t kNoAllocSlotsCap = dense_slots_cap(kNoAllocMaxN);
constexpr size_t kNoAllocItems = ((size_t)kNoAllocItemsCap * sizeof(int4) + 255) / 256 * 256;
constexpr size_t kNoAllocPartial =
    ((size_t)kNoAllocSlotsCap * (PMMM_PMAX + 1) * (PMMM_PMAX + 1 + 1) * sizeof(float) + 255) /
    256 * 256;
constexpr size_t kNoAllocBytes = 5 * kNoAllocInts + 2 * kNoAllocRecs + kNoAllocHist +
                                 kNoAllocSums + kNoAllocItems + kNoAllocPartial;
static_assert(kNoAllocInts % 256 == 0 && kNoAllocRecs % 256 == 0 && kNoAllocHist % 256 == 0,
              "256-byte aligned regions");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of each GPU's copy of `scratch`, looked up once per device
// (with that device current); host code uses these, never the array's name.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {nullptr};

static int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the library's table of devices");
        return PMMM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device] != nullptr) return PMMM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = ptr;
    return PMMM_OK;
}

static int far_noalloc(pmmm_plan_s *pl, int64_t n, const float *x, const float *y,
                       const float *z, const float *q, float *phi, float *gx, float *gy,
                       float *gz, void *stream) {
    if (!pl) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    if (pl->tsize != sizeof(float)) {
        set_error("pmmm_far_f32_noalloc needs a PMMM_F32 or PMMM_BF16X3 plan");
        return PMMM_EINVAL;
    }
    if (n < 0 || n > kNoAllocMaxN) {
        set_error("n outside 0..PMMM_NOALLOC_MAX_N, the capacity of the static scratch");
        return PMMM_EINVAL;
    }
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (pl->device >= 0 && pl->device < kMaxDevices) base = g_scratch_dev[pl->device];
    }
    if (base == nullptr) {
        set_error("static scratch of the plan's device not set up");
        return PMMM_EHIP;
    }
    unsigned char *b = (unsigned char *)base;
    PBuf pb{};
    pb.cell_of = (int *)(b);
    pb.slot = (int *)(b + kNoAllocInts);
    pb.perm = (int *)(b + 2 * kNoAllocInts);
    pb.scell = (int *)(b + 3 * kNoAllocInts);
    pb.pos = (int *)(b + 4 * kNoAllocInts);
    pb.sorted = b + 5 * kNoAllocInts;
    pb.staged = b + 5 * kNoAllocInts + kNoAllocRecs;
    pb.count = (int *)(b + 5 * kNoAllocInts + 2 * kNoAllocRecs);
    pb.tile_sums = (int *)(b + 5 * kNoAllocInts + 2 * kNoAllocRecs + kNoAllocHist);
    pb.items = (int4 *)(b + 5 * kNoAllocInts + 2 * kNoAllocRecs + kNoAllocHist + kNoAllocSums);
    pb.partial = (float *)(b + 5 * kNoAllocInts + 2 * kNoAllocRecs + kNoAllocHist +
                           kNoAllocSums + kNoAllocItems);
    pb.items_cap = kNoAllocItemsCap;
    pb.slots_cap = kNoAllocSlotsCap;
    pb.tile_row = nullptr;  // far field only
    if ((size_t)bin_hist_ints(n) * sizeof(int) > kNoAllocHist ||
        (size_t)bin_scan_tiles(n) * sizeof(int) > kNoAllocSums) {
        set_error("radix-sort scratch exceeds the static array");
        return PMMM_EINVAL;
    }
    return call_impl<float>(pl, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, stream, &pb);
}

static int ensure_multi(Plan *pl, int sets, hipStream_t s) {
    if (pl->mtmap == nullptr) {
        std::vector<unsigned> map(multi_map_entries(pl->p));
        build_multi_map(pl->p, map.data());
        PMMM_HIP(hipMalloc(&pl->mtmap, map.size() * sizeof(unsigned)));
        PMMM_HIP(hipMemcpyAsync(pl->mtmap, map.data(), map.size() * sizeof(unsigned),
                                hipMemcpyHostToDevice, s));
        PMMM_HIP(hipStreamSynchronize(s));
    }
    if (sets <= pl->mcap_sets) return PMMM_OK;
    PMMM_HIP(hipDeviceSynchronize());
    hipFree(pl->mM);
    hipFree(pl->mY);
    hipFree(pl->mqr2);
    hipFree(pl->mqtot);
    pl->mM = nullptr;
    pl->mY = nullptr;
    pl->mqr2 = pl->mqtot = nullptr;
    pl->mcap_sets = 0;
    const size_t P = pl->P, K = pl->K;
    PMMM_HIP(hipMalloc(&pl->mM, (size_t)sets * (P + 1) * K * sizeof(float)));
    // spectra: one slice of P sets complex values (padded to even) per frequency
    PMMM_HIP(hipMalloc(&pl->mY, ((size_t)sets * P + 1) * pl->nf * pl->ncol * 2 * sizeof(float)));
    PMMM_HIP(hipMalloc(&pl->mqr2, (size_t)sets * pl->nf * sizeof(double)));
    PMMM_HIP(hipMalloc(&pl->mqtot, (size_t)sets * sizeof(double)));
    pl->mcap_sets = sets;
    return PMMM_OK;
}

static int multi_impl(pmmm_plan_s *pl, int64_t n, const float *x, const float *y,
                      const float *z, int nsets, const float *q, float *phi, float *gx,
                      float *gy, float *gz, void *stream) {
    if (!pl) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    if (pl->tsize != sizeof(float)) {
        set_error("multi-charge calls need a PMMM_F32 or PMMM_BF16X3 plan");
        return PMMM_EINVAL;
    }
    if (n < 0 || nsets < 1) {
        set_error("n must be non-negative and nsets positive");
        return PMMM_EINVAL;
    }
    if (n > 0 && (!x || !y || !z || !q || !phi || !gx || !gy || !gz)) {
        set_error("NULL particle or output pointer");
        return PMMM_EINVAL;
    }
    if (pl->open || !multi_supported(pl->p, pl->nf)) {
        set_error("multi-charge calls are built for periodic meshes of 4, 8, 16 or 32 cells "
                  "per axis and orders p <= 8");
        return PMMM_EUNSUPPORTED;
    }
    const int split = pl->prec == PMMM_BF16X3 ? 2 : 3;
    const int chunk = nsets < kMultiMaxSets ? nsets : kMultiMaxSets;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    PMMM_HIP(hipGetDevice(&cur));
    if (cur != pl->device) {
        set_error("current device differs from the plan's device");
        return PMMM_EINVAL;
    }
    int rc = ensure_capacity(pl, n > 0 ? n : 1);
    if (rc != PMMM_OK) return rc;
    rc = ensure_multi(pl, chunk, s);
    if (rc != PMMM_OK) return rc;
    pl->last_stream = s;
    pl->last_n = n;
    {
        StageTimer t(pl, PMMM_STAGE_BIN, s);
        BinArgs b{};
        b.n = n;
        b.x = x;
        b.y = y;
        b.z = z;
        b.q = nullptr;            // sorted charges stay zero; the sets are read by P2M
        b.ncell = pl->n;
        b.inv_h = pl->inv_h;
        b.periodic = 1;
        b.cell_of = pl->cell_of;
        b.slot = pl->slot;
        b.count = pl->count;
        b.start = pl->start;
        b.scell = pl->scell;
        b.perm = pl->perm;
        b.flag = pl->small + 1;
        b.items = nullptr;        // the multi-charge P2M reduces every cell itself
        b.small = pl->small;
        b.tile_sums = pl->tile_sums;
        b.sorted = pl->sorted;
        b.recs = pl->staged;
        PMMM_HIP(launch_bin<float>(b, s));
    }
    for (int s0 = 0; s0 < nsets; s0 += kMultiMaxSets) {
        const int S = nsets - s0 < kMultiMaxSets ? nsets - s0 : kMultiMaxSets;
        MultiArgs a{};
        a.p = pl->p;
        a.n = pl->n;
        a.nsets = S;
        a.split = split;
        a.np = n;
        a.ld = nsets;
        a.start = pl->start;
        a.perm = pl->perm;
        a.zero_count = nullptr;
        a.sorted = pl->sorted;
        a.q = q + s0;
        a.M = pl->mM;
        a.Y = pl->mY;
        a.green = (const float *)pl->green;
        a.tw = pl->tw;
        a.tmap = pl->mtmap;
        a.qr2_partial = pl->mqr2;
        a.qtot = pl->mqtot;
        a.alpha_cell = pl->alpha_cell;
        a.inv_h = pl->inv_h;
        a.phi = phi + s0;
        a.gx = gx + s0;
        a.gy = gy + s0;
        a.gz = gz + s0;
        static const int stage_of[5] = {PMMM_STAGE_P2M, PMMM_STAGE_FFT_FWD, PMMM_STAGE_COLUMN,
                                        PMMM_STAGE_FFT_INV, PMMM_STAGE_L2P};
        for (int st = 0; st < 5; ++st) {
            StageTimer t(pl, stage_of[st], s);
            PMMM_HIP(launch_multi_stage(a, st, s));
        }
    }
    return PMMM_OK;
}

// Shortest event time (ms) of one stage over `reps` far-field calls with the
// plan's current launch shapes (after one untimed call).
template <typename T>
static int time_stage(pmmm_plan_s *pl, int stage, int reps, int64_t n, const T *x, const T *y,
                      const T *z, const T *q, T *phi, T *gx, T *gy, T *gz, hipStream_t s,
                      float *best_ms) {
    int rc = call_impl<T>(pl, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, s);
    pl->prof_mask = 1u << stage;
    for (int it = 0; it < reps && rc == PMMM_OK; ++it)
        rc = call_impl<T>(pl, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, s);
    pl->prof_mask = 0;
    float mn = 1e30f;
    for (auto &pr : pl->ev_pending[stage]) {
        float t = 1e30f;
        if (hipEventSynchronize(pr.second) == hipSuccess &&
            hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess)
            mn = t < mn ? t : mn;
        pl->ev_pool.push_back(pr.first);
        pl->ev_pool.push_back(pr.second);
    }
    pl->ev_pending[stage].clear();
    *best_ms = mn;
    return rc;
}

// Autotuner: on the caller's particles, times the P2M stage for each number
// of lanes per cell (4..32) and then the column stage for each column-kernel
// width w (the widest that fits down to a quarter of it), each candidate in
// three interleaved rounds, and keeps the fastest of each.
template <typename T>
static int autotune_impl(pmmm_plan_s *pl, int64_t n, const T *x, const T *y, const T *z,
                         const T *q, T *phi, T *gx, T *gy, T *gz, hipStream_t s) {
    // column candidates: (form, width)
    std::vector<std::pair<int, int>> cand;
    if (pl->generic) {
        cand.push_back({0, 0});     // one M2L kernel, no forms to choose from
    } else {
        int wmax = 1, rs = 1;
        if (column_shape(pl->p, pl->nf, pl->tsize, &wmax, &rs) > 0) {
            cand.push_back({PMMM_COLUMN_TILE, wmax});
            if (wmax >= 2) cand.push_back({PMMM_COLUMN_TILE, wmax / 2});
            if (wmax >= 4) cand.push_back({PMMM_COLUMN_TILE, wmax / 4});
        }
        for (int kind : {PMMM_COLUMN_STREAM_1, PMMM_COLUMN_STREAM_2, PMMM_COLUMN_STREAM_4})
            if (column_kernel_fits(kind, pl->p, pl->nf, pl->tsize)) cand.push_back({kind, 0});
    }
    if (cand.empty()) return PMMM_EUNSUPPORTED;
    const int gs[4] = {4, 8, 16, 32};
    constexpr int kRounds = 3, kReps = 5;
    // the caller's own stage profiling (if any) is set aside meanwhile
    int rc = pmmm_plan_read_profile(pl, nullptr, nullptr, 0);
    if (rc != PMMM_OK) return rc;
    const unsigned mask = pl->prof_mask;
    float tg[4] = {1e30f, 1e30f, 1e30f, 1e30f};
    std::vector<float> tw(cand.size(), 1e30f);
    pl->tune_col_kernel = 0;
    pl->tune_col_w = 0;
    for (int r = 0; r < kRounds && rc == PMMM_OK; ++r) {
        for (int k = 0; k < 4 && rc == PMMM_OK; ++k) {
            pl->tune_group = gs[k];
            float t = 0.f;
            rc = time_stage<T>(pl, PMMM_STAGE_P2M, kReps, n, x, y, z, q, phi, gx, gy, gz, s, &t);
            tg[k] = t < tg[k] ? t : tg[k];
        }
    }
    int bg = 0;
    for (int k = 1; k < 4; ++k)
        if (tg[k] < tg[bg]) bg = k;
    pl->tune_group = gs[bg];
    for (int r = 0; r < kRounds && rc == PMMM_OK; ++r) {
        for (size_t k = 0; k < cand.size() && rc == PMMM_OK; ++k) {
            pl->tune_col_kernel = cand[k].first;
            pl->tune_col_w = cand[k].second;
            float t = 0.f;
            rc = time_stage<T>(pl, PMMM_STAGE_COLUMN, kReps, n, x, y, z, q, phi, gx, gy, gz, s, &t);
            tw[k] = t < tw[k] ? t : tw[k];
        }
    }
    size_t bw = 0;
    for (size_t k = 1; k < cand.size(); ++k)
        if (tw[k] < tw[bw]) bw = k;
    pl->prof_mask = mask;
    pl->tune_col_kernel = rc == PMMM_OK ? cand[bw].first : 0;
    pl->tune_col_w = rc == PMMM_OK ? cand[bw].second : 0;
    pl->tune_group = rc == PMMM_OK ? gs[bg] : 0;
    return rc;
}

// ------------------------------------------------------------------ batches
// Systems with equal method parameters (mesh, box, order, cutoff, boundary,
// splitting, images) form a class: one transfer kernel, one launch per stage
// for all of them (blockIdx.y / .z selects the system), per-system meshes at
// fixed strides in the class workspace.
struct BatchClass {
    pmmm_plan_s *plan = nullptr;    // transfer kernel, twiddles, constants
    std::vector<int> members;       // system indices in the caller's order
    int *start = nullptr, *small = nullptr;
    int *count = nullptr, *tile_sums = nullptr;   // radix-sort scratch, sized by max_np
    int4 *items = nullptr;          // dense P2M items, [ns][items_cap]
    float *partial = nullptr;       // [ns][slots_cap][P + 1]
    int64_t hist_cap = -1;          // max_np the radix scratch and the items hold
    int64_t items_cap = 0, slots_cap = 0;
    void *M = nullptr, *spec = nullptr, *L = nullptr;
    double *qr2 = nullptr, *sums = nullptr;
    int64_t *d_prange = nullptr;    // [2 members]
    int64_t max_np = 0, tot_np = 0;
};

struct pmmm_batch_s {
    int nsys = 0, device = 0;
    std::vector<BatchClass> cls;
    int64_t cap = 0;
    int *cell_of = nullptr, *slot = nullptr, *perm = nullptr, *scell = nullptr;
    void *sorted = nullptr, *recs = nullptr;
    int *flag = nullptr;
    int64_t *h_prange = nullptr;    // pinned staging [2 nsys]
    std::vector<int64_t> offsets;   // of the last call
    hipStream_t last_stream = nullptr;
    // the last call's launches as a graph, replayed while the arguments repeat
    int use_graph = 1;
    std::vector<const void *> key;
    int key_hits = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // classes run concurrently on side streams (default priority), forked
    // from and joined back into the caller's stream with events
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    std::vector<int> lane_of;       // side stream of each class (longest first, least loaded)
};

// Side streams of a batch: classes are independent (disjoint particle
// ranges, their own meshes), so up to this many run at once.
constexpr int kBatchStreams = 4;

static bool same_class(const pmmm_params &a, const pmmm_params &b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.box[0] == b.box[0] &&
           a.box[1] == b.box[1] && a.box[2] == b.box[2] && a.p == b.p &&
           (a.cutoff == 0 ? 2 : a.cutoff) == (b.cutoff == 0 ? 2 : b.cutoff) &&
           a.boundary == b.boundary && a.alpha == b.alpha && a.images == b.images;
}

static void drop_graph(pmmm_batch_s *b) {
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->key.clear();
    b->key_hits = 0;
}

static void batch_destroy(pmmm_batch_s *b) {
    if (!b) return;
    hipDeviceSynchronize();
    drop_graph(b);
    for (auto &c : b->cls) {
        hipFree(c.count);
        hipFree(c.start);
        hipFree(c.items);
        hipFree(c.partial);
        hipFree(c.tile_sums);
        hipFree(c.small);
        hipFree(c.M);
        hipFree(c.spec);
        hipFree(c.L);
        hipFree(c.qr2);
        hipFree(c.sums);
        hipFree(c.d_prange);
        destroy(c.plan);
    }
    hipFree(b->cell_of);
    hipFree(b->slot);
    hipFree(b->perm);
    hipFree(b->scell);
    hipFree(b->sorted);
    hipFree(b->recs);
    hipFree(b->flag);
    if (b->h_prange) hipHostFree(b->h_prange);
    for (hipStream_t st : b->side) hipStreamDestroy(st);
    for (hipEvent_t ev : b->join) hipEventDestroy(ev);
    if (b->fork) hipEventDestroy(b->fork);
    delete b;
}

static int batch_alloc_class(BatchClass &c, hipStream_t s) {
    const Plan *pl = c.plan;
    const size_t ns = c.members.size(), K = pl->K, P = pl->P, t = pl->tsize;
    PMMM_HIP(hipMalloc(&c.start, sizeof(int) * (K + 1) * ns));
    PMMM_HIP(hipMalloc(&c.small, sizeof(int) * 8 * ns));
    PMMM_HIP(hipMalloc(&c.M, t * (P + 1) * K * ns));
    PMMM_HIP(hipMalloc(&c.spec, 2 * t * P * pl->n * pl->ncol * ns));
    PMMM_HIP(hipMalloc(&c.L, t * P * K * ns));
    PMMM_HIP(hipMalloc(&c.qr2, sizeof(double) * pl->n * ns));
    PMMM_HIP(hipMalloc(&c.sums, sizeof(double) * 8 * ns));
    PMMM_HIP(hipMalloc(&c.d_prange, sizeof(int64_t) * 2 * ns));
    PMMM_HIP(hipMemsetAsync(c.small, 0, sizeof(int) * 8 * ns, s));
    PMMM_HIP(hipMemsetAsync(c.M, 0, t * (P + 1) * K * ns, s));
    return PMMM_OK;
}

static int batch_capacity(pmmm_batch_s *b, int64_t n) {
    if (n <= b->cap) return PMMM_OK;
    if (n > (int64_t)INT32_MAX) {
        set_error("particle count exceeds the 32-bit index range");
        return PMMM_EINVAL;
    }
    PMMM_HIP(hipDeviceSynchronize());
    drop_graph(b);
    hipFree(b->cell_of);
    hipFree(b->slot);
    hipFree(b->perm);
    hipFree(b->scell);
    hipFree(b->sorted);
    hipFree(b->recs);
    b->sorted = b->recs = nullptr;
    b->cap = 0;
    PMMM_HIP(hipMalloc(&b->cell_of, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&b->slot, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&b->perm, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&b->scell, sizeof(int) * n));
    PMMM_HIP(hipMalloc(&b->sorted, sizeof(float) * 4 * n));
    PMMM_HIP(hipMalloc(&b->recs, sizeof(float) * 4 * n));
    b->cap = n;
    return PMMM_OK;
}

// Every launch of one batched far-field call, class by class.
static int class_enqueue(pmmm_batch_s *b, BatchClass &c, const float *x, const float *y,
                         const float *z, const float *q, float *phi, float *gx, float *gy,
                         float *gz, hipStream_t s) {
    {
        const Plan *pl = c.plan;
        const int ns = (int)c.members.size();
        const int group = group_for((double)c.tot_np / ((double)pl->K * ns));
        const int dense_thr = dense_threshold_for(group);
        BinArgs bn{};
        bn.n = 0;
        bn.x = x;
        bn.y = y;
        bn.z = z;
        bn.q = q;
        bn.ncell = pl->n;
        bn.inv_h = pl->inv_h;
        bn.periodic = !pl->open;
        for (int a3 = 0; a3 < 3; ++a3) bn.lim[a3] = pl->lim[a3];
        bn.cell_of = b->cell_of;
        bn.slot = b->slot;
        bn.count = c.count;
        bn.start = c.start;
        bn.scell = b->scell;
        bn.perm = b->perm;
        bn.flag = b->flag;
        bn.items = c.items;
        bn.items_cap = c.items_cap;
        bn.slots_cap = c.slots_cap;
        bn.small = c.small;
        bn.tile_sums = c.tile_sums;
        bn.dense_threshold = dense_thr;
        bn.sorted = b->sorted;
        bn.recs = b->recs;
        bn.prange = c.d_prange;
        bn.nsys = ns;
        bn.max_np = c.max_np;
        PMMM_HIP(launch_bin<float>(bn, s));
        P2MArgs m{};
        m.p = pl->p;
        m.ncell = pl->n;
        m.group = group;
        m.start = c.start;
        m.dense_threshold = dense_thr;
        m.items = c.items;
        m.items_cap = c.items_cap;
        m.small = c.small;
        m.partial = c.partial;
        m.slots_cap = c.slots_cap;
        m.sorted = b->sorted;
        m.M = c.M;
        m.prange = c.d_prange;
        m.nsys = ns;
        PMMM_HIP(launch_p2m<float>(m, s));
        FFTArgs f{};
        f.p = pl->p;
        f.n = pl->n;
        f.nf = pl->nf;
        f.open = pl->open;
        f.M = c.M;
        f.spec = c.spec;
        f.green = pl->green;
        f.tw = pl->tw;
        f.L = c.L;
        f.qr2_partial = c.qr2;
        f.sums = c.sums;
        f.nsys = ns;
        for (int st = 0; st < 3; ++st) PMMM_HIP(launch_conv_stage<float>(f, st, s));
        L2PArgs l{};
        l.n = 0;
        l.p = pl->p;
        l.ncell = pl->n;
        l.periodic = !pl->open;
        l.sorted = b->sorted;
        l.scell = b->scell;
        l.perm = b->perm;
        l.L = c.L;
        l.sums = c.sums;
        l.alpha_cell = pl->alpha_cell;
        l.inv_h = pl->inv_h;
        l.phi = phi;
        l.gx = gx;
        l.gy = gy;
        l.gz = gz;
        l.prange = c.d_prange;
        l.nsys = ns;
        l.max_np = c.max_np;
        PMMM_HIP(launch_l2p<float>(l, s));
    }
    return PMMM_OK;
}

// Assign the classes to the side streams, longest first to the least loaded
// (work ~ particles x expansion terms + mesh x terms).
static void batch_plan_lanes(pmmm_batch_s *b) {
    const int nl = (int)b->side.size();
    b->lane_of.assign(b->cls.size(), 0);
    if (nl < 2) return;
    std::vector<int> order(b->cls.size());
    std::vector<double> cost(b->cls.size()), load(nl, 0.0);
    for (size_t i = 0; i < b->cls.size(); ++i) {
        const BatchClass &c = b->cls[i];
        order[i] = (int)i;
        cost[i] = ((double)c.tot_np + 4.0 * (double)c.plan->K * c.members.size()) * c.plan->P;
    }
    std::sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    for (int i : order) {
        int best = 0;
        for (int k = 1; k < nl; ++k)
            if (load[k] < load[best]) best = k;
        load[best] += cost[i];
        b->lane_of[i] = best;
    }
}

// Every launch of one batched far-field call: the classes on the side
// streams, forked from and joined back into s (also under graph capture,
// where the fork and join events make them parallel branches).
static int batch_enqueue(pmmm_batch_s *b, const float *x, const float *y, const float *z,
                         const float *q, float *phi, float *gx, float *gy, float *gz,
                         hipStream_t s) {
    if (b->side.size() < 2 || b->cls.size() < 2) {
        for (auto &c : b->cls) {
            const int rc = class_enqueue(b, c, x, y, z, q, phi, gx, gy, gz, s);
            if (rc != PMMM_OK) return rc;
        }
        return PMMM_OK;
    }
    if (b->lane_of.size() != b->cls.size()) batch_plan_lanes(b);
    PMMM_HIP(hipEventRecord(b->fork, s));
    for (hipStream_t st : b->side) PMMM_HIP(hipStreamWaitEvent(st, b->fork, 0));
    for (size_t i = 0; i < b->cls.size(); ++i) {
        const int rc = class_enqueue(b, b->cls[i], x, y, z, q, phi, gx, gy, gz,
                                     b->side[b->lane_of[i]]);
        if (rc != PMMM_OK) return rc;
    }
    for (size_t k = 0; k < b->side.size(); ++k) {
        PMMM_HIP(hipEventRecord(b->join[k], b->side[k]));
        PMMM_HIP(hipStreamWaitEvent(s, b->join[k], 0));
    }
    return PMMM_OK;
}

static int batch_far(pmmm_batch_s *b, const int64_t *offsets, const float *x, const float *y,
                     const float *z, const float *q, float *phi, float *gx, float *gy,
                     float *gz, void *stream) {
    if (!b || !offsets) {
        set_error("NULL batch or offsets");
        return PMMM_EINVAL;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return PMMM_EINVAL;
    }
    for (int i = 0; i < b->nsys; ++i) {
        if (offsets[i + 1] < offsets[i]) {
            set_error("offsets must be non-decreasing");
            return PMMM_EINVAL;
        }
    }
    const int64_t total = offsets[b->nsys];
    if (total > 0 && (!x || !y || !z || !q || !phi || !gx || !gy || !gz)) {
        set_error("NULL particle or output pointer");
        return PMMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    PMMM_HIP(hipGetDevice(&cur));
    if (cur != b->device) {
        set_error("current device differs from the batch's device");
        return PMMM_EINVAL;
    }
    int rc = batch_capacity(b, total > 0 ? total : 1);
    if (rc != PMMM_OK) return rc;
    b->last_stream = s;
    if (b->offsets.size() != (size_t)b->nsys + 1 ||
        !std::equal(b->offsets.begin(), b->offsets.end(), offsets)) {
        // new particle ranges: restage them for every class (pinned buffer,
        // synchronised before it is reused)
        drop_graph(b);
        PMMM_HIP(hipStreamSynchronize(s));
        int64_t *h = b->h_prange;
        for (auto &c : b->cls) {
            c.max_np = 0;
            c.tot_np = 0;
            for (size_t k = 0; k < c.members.size(); ++k) {
                const int m = c.members[k];
                h[2 * k] = offsets[m];
                h[2 * k + 1] = offsets[m + 1];
                const int64_t np = offsets[m + 1] - offsets[m];
                c.max_np = np > c.max_np ? np : c.max_np;
                c.tot_np += np;
            }
            PMMM_HIP(hipMemcpyAsync(c.d_prange, h, sizeof(int64_t) * 2 * c.members.size(),
                                    hipMemcpyHostToDevice, s));
            PMMM_HIP(hipStreamSynchronize(s));
            if (c.count == nullptr || bin_hist_ints(c.max_np) > bin_hist_ints(c.hist_cap)) {
                // radix-sort scratch for the largest system of the class
                const size_t ns = c.members.size();
                hipFree(c.count);
                hipFree(c.tile_sums);
                hipFree(c.items);
                hipFree(c.partial);
                c.count = c.tile_sums = nullptr;
                c.items = nullptr;
                c.partial = nullptr;
                c.hist_cap = -1;
                const int64_t ic = dense_items_cap(c.max_np, c.plan->K);
                const int64_t sc = dense_slots_cap(c.max_np);
                PMMM_HIP(hipMalloc(&c.count, sizeof(int) * bin_hist_ints(c.max_np) * ns));
                PMMM_HIP(hipMalloc(&c.tile_sums, sizeof(int) * bin_scan_tiles(c.max_np) * ns));
                PMMM_HIP(hipMalloc(&c.items, sizeof(int4) * ic * ns));
                PMMM_HIP(hipMalloc(&c.partial, sizeof(float) * sc * (c.plan->P + 1) * ns));
                c.items_cap = ic;
                c.slots_cap = sc;
                c.hist_cap = c.max_np;
            }
        }
        b->offsets.assign(offsets, offsets + b->nsys + 1);
        b->lane_of.clear();   // the classes' loads changed: reassign their streams
    }
    const std::vector<const void *> key = {x, y, z, q, phi, gx, gy, gz, (const void *)s};
    const bool graphs = b->use_graph && s != nullptr;
    if (graphs && key == b->key) {
        if (b->gexec == nullptr) {
            // second call with these arguments: capture the launches once
            PMMM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            rc = batch_enqueue(b, x, y, z, q, phi, gx, gy, gz, s);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &g);
            if (rc != PMMM_OK) {
                if (g) hipGraphDestroy(g);
                return rc;
            }
            PMMM_HIP(e);
            b->graph = g;
            PMMM_HIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
        }
        PMMM_HIP(hipGraphLaunch(b->gexec, s));
        return PMMM_OK;
    }
    drop_graph(b);
    b->key = key;
    return batch_enqueue(b, x, y, z, q, phi, gx, gy, gz, s);
}

// ------------------------------------------------ two-level hierarchy
struct pmmm_hier_s {
    pmmm_plan_s *coarse = nullptr, *fine = nullptr;
    float *table = nullptr;
};

static void hier_destroy(pmmm_hier_s *h) {
    if (!h) return;
    if (h->coarse) destroy(h->coarse);
    if (h->fine) destroy(h->fine);
    if (h->table) hipFree(h->table);
    delete h;
}

// The fine plan: binning, P2M, L2P and the near field on the refined mesh,
// no transfer kernel or spectra.
static int fine_plan_create(const pmmm_params *coarse, int r, hipStream_t s, pmmm_plan_s **out) {
    pmmm_params fp = *coarse;
    fp.nx = fp.ny = fp.nz = coarse->nx * r;
    pmmm_plan_s *pl = new pmmm_plan_s();
    derive(pl, &fp);
    pl->no_transfer = true;
    hipError_t e = hipGetDevice(&pl->device);
    int rc = e == hipSuccess ? PMMM_OK : hip_fail(e, "hipGetDevice");
    if (rc == PMMM_OK) rc = alloc_plan(pl, s);
    if (rc == PMMM_OK) rc = scratch_setup(pl->device);
    if (rc == PMMM_OK && fp.n_max > 0) rc = ensure_capacity(pl, fp.n_max);
    if (rc != PMMM_OK) {
        destroy(pl);
        return rc;
    }
    *out = pl;
    return PMMM_OK;
}

extern "C" {

int pmmm_hier_create(const pmmm_params *coarse, int refine, void *stream, pmmm_hier *out) {
    if (!out) {
        set_error("out is NULL");
        return PMMM_EINVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = validate(coarse, why);
    if (rc != PMMM_OK) {
        set_error(why);
        return rc;
    }
    if (coarse->boundary != PMMM_OPEN || coarse->precision != PMMM_F32 || coarse->nx != coarse->ny ||
        coarse->nx != coarse->nz || !is_pow2(coarse->nx)) {
        set_error("the hierarchy takes an open FP32 coarse mesh, cubic with a power-of-two edge");
        return PMMM_EUNSUPPORTED;
    }
    if (refine != 1 && refine != 2 && refine != 4 && refine != 8) {
        set_error("refine must be 1, 2, 4 or 8");
        return PMMM_EINVAL;
    }
    if (coarse->nx * refine > 128) {
        set_error("the fine mesh is limited to 128 cells per axis");
        return PMMM_EUNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    pmmm_hier_s *h = new pmmm_hier_s();
    rc = pmmm_plan_create(coarse, stream, &h->coarse);
    if (rc == PMMM_OK) rc = fine_plan_create(coarse, refine, s, &h->fine);
    if (rc == PMMM_OK) {
        const int c = h->fine->cutoff, D = (c + 1) * refine - 1, W = 2 * D + 1;
        const size_t bytes = sizeof(float) * (size_t)W * W * W * h->fine->Q;
        hipError_t e = hipMalloc(&h->table, bytes);
        if (e == hipSuccess) e = build_hier_table_f32(h->fine->p, c, D, h->table, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "hierarchy table");
        } else {
            h->fine->hier_table = h->table;
            h->fine->hier_r = refine;
            h->fine->hier_D = D;
        }
    }
    if (rc != PMMM_OK) {
        hier_destroy(h);
        return rc;
    }
    *out = h;
    return PMMM_OK;
}

void pmmm_hier_destroy(pmmm_hier h) { hier_destroy(h); }

int pmmm_hier_far_f32(pmmm_hier h, int64_t n, const float *x, const float *y, const float *z,
                      const float *q, float *phi, float *gx, float *gy, float *gz, void *stream) {
    if (!h) {
        set_error("hierarchy is NULL");
        return PMMM_EINVAL;
    }
    int rc = call_impl<float>(h->coarse, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
    if (rc != PMMM_OK || n == 0) return rc;
    return call_impl<float>(h->fine, kHierFine, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_hier_total_f32(pmmm_hier h, int64_t n, const float *x, const float *y, const float *z,
                        const float *q, float *phi, float *gx, float *gy, float *gz, void *stream) {
    if (!h) {
        set_error("hierarchy is NULL");
        return PMMM_EINVAL;
    }
    int rc = call_impl<float>(h->coarse, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
    if (rc != PMMM_OK || n == 0) return rc;
    return call_impl<float>(h->fine, kHierTotal, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_hier_set_profiling(pmmm_hier h, unsigned mask) {
    if (!h) {
        set_error("hierarchy is NULL");
        return PMMM_EINVAL;
    }
    const int rc = pmmm_plan_set_profiling(h->coarse, mask);
    return rc != PMMM_OK ? rc : pmmm_plan_set_profiling(h->fine, mask);
}

int pmmm_hier_read_profile(pmmm_hier h, int level, double *ms, int64_t *count, int reset) {
    if (!h || (level != 0 && level != 1)) {
        set_error(!h ? "hierarchy is NULL" : "level must be 0 (coarse) or 1 (fine)");
        return PMMM_EINVAL;
    }
    return pmmm_plan_read_profile(level == 0 ? h->coarse : h->fine, ms, count, reset);
}

int pmmm_hier_sync_status(pmmm_hier h) {
    if (!h) {
        set_error("hierarchy is NULL");
        return PMMM_EINVAL;
    }
    const int rc = pmmm_plan_sync_status(h->coarse);
    const int rf = pmmm_plan_sync_status(h->fine);
    return rc != PMMM_OK ? rc : rf;
}

}  // extern "C"

extern "C" {

int pmmm_plan_create(const pmmm_params *params, void *stream, pmmm_plan *out) {
    if (!out) {
        set_error("out is NULL");
        return PMMM_EINVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = validate(params, why);
    if (rc != PMMM_OK) {
        set_error(why);
        return rc;
    }
    pmmm_plan_s *pl = new pmmm_plan_s();
    derive(pl, params);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&pl->device);
    if (e != hipSuccess) {
        rc = hip_fail(e, "hipGetDevice");
        destroy(pl);
        return rc;
    }
    rc = alloc_plan(pl, s);
    if (rc == PMMM_OK) rc = scratch_setup(pl->device);
    if (rc == PMMM_OK && params->n_max > 0) rc = ensure_capacity(pl, params->n_max);
    if (rc == PMMM_OK) {
        GreenArgs g{};
        g.p = pl->p;
        g.n = pl->n;
        g.nf = pl->nf;
        g.open = pl->open;
        g.cutoff = pl->cutoff;
        g.images = pl->images;
        g.alpha_cell = pl->alpha_cell;
        g.green_out = pl->green;
        e = pl->prec == PMMM_F64 ? build_green<double>(g, s) : build_green<float>(g, s);
        if (e != hipSuccess) rc = hip_fail(e, "transfer kernel build");
    }
    if (rc != PMMM_OK) {
        destroy(pl);
        return rc;
    }
    *out = pl;
    return PMMM_OK;
}

void pmmm_plan_destroy(pmmm_plan plan) { destroy(plan); }

size_t pmmm_workspace_bytes(const pmmm_params *params, int64_t n_max) {
    std::string why;
    if (validate(params, why) != PMMM_OK || n_max < 0) return 0;
    Plan pl;
    derive(&pl, params);
    return plan_bytes(&pl) + particle_bytes(&pl, n_max);
}

int pmmm_far_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                 const float *q, float *phi, float *gx, float *gy, float *gz, void *stream) {
    return call_impl<float>(plan, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_far_f64(pmmm_plan plan, int64_t n, const double *x, const double *y, const double *z,
                 const double *q, double *phi, double *gx, double *gy, double *gz,
                 void *stream) {
    return call_impl<double>(plan, kFar, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_far_f32_noalloc(pmmm_plan plan, int64_t n, const float *x, const float *y,
                         const float *z, const float *q, float *phi, float *gx, float *gy,
                         float *gz, void *stream) {
    return far_noalloc(plan, n, x, y, z, q, phi, gx, gy, gz, stream);
}

int pmmm_total_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                   const float *q, float *phi, float *gx, float *gy, float *gz, void *stream) {
    return call_impl<float>(plan, kTotal, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_total_f64(pmmm_plan plan, int64_t n, const double *x, const double *y,
                   const double *z, const double *q, double *phi, double *gx, double *gy,
                   double *gz, void *stream) {
    return call_impl<double>(plan, kTotal, n, x, y, z, q, phi, gx, gy, gz, 0, stream);
}

int pmmm_far_multi_f32(pmmm_plan plan, int64_t n, const float *x, const float *y,
                       const float *z, int nsets, const float *q, float *phi, float *gx,
                       float *gy, float *gz, void *stream) {
    return multi_impl(plan, n, x, y, z, nsets, q, phi, gx, gy, gz, stream);
}

int pmmm_near_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                  const float *q, float *phi, float *gx, float *gy, float *gz, int accumulate,
                  void *stream) {
    return call_impl<float>(plan, kNear, n, x, y, z, q, phi, gx, gy, gz, accumulate, stream);
}

int pmmm_near_f64(pmmm_plan plan, int64_t n, const double *x, const double *y,
                  const double *z, const double *q, double *phi, double *gx, double *gy,
                  double *gz, int accumulate, void *stream) {
    return call_impl<double>(plan, kNear, n, x, y, z, q, phi, gx, gy, gz, accumulate, stream);
}

int pmmm_batch_create(int nsys, const pmmm_params *per_sys, void *stream, pmmm_batch *out) {
    if (!out) {
        set_error("out is NULL");
        return PMMM_EINVAL;
    }
    *out = nullptr;
    if (nsys < 1 || !per_sys) {
        set_error("nsys must be positive and per_sys non-NULL");
        return PMMM_EINVAL;
    }
    for (int i = 0; i < nsys; ++i) {
        std::string why;
        const int rc = validate(&per_sys[i], why);
        if (rc != PMMM_OK) {
            set_error("system " + std::to_string(i) + ": " + why);
            return rc;
        }
        if (per_sys[i].precision == PMMM_F64) {
            set_error("batches run the FP32 pipeline (PMMM_F32 or PMMM_BF16X3 systems)");
            return PMMM_EINVAL;
        }
        if (per_sys[i].boundary == PMMM_PERIODIC && !is_pow2(per_sys[i].nx)) {
            set_error("system " + std::to_string(i) +
                      ": batches take periodic meshes of power-of-two edge only");
            return PMMM_EUNSUPPORTED;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    pmmm_batch_s *b = new pmmm_batch_s();
    b->nsys = nsys;
    int rc = PMMM_OK;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) rc = hip_fail(e, "hipGetDevice");
    for (int i = 0; i < nsys && rc == PMMM_OK; ++i) {
        size_t k = 0;
        while (k < b->cls.size() && !same_class(b->cls[k].plan->prm, per_sys[i])) ++k;
        if (k == b->cls.size()) {
            BatchClass c;
            pmmm_params prm = per_sys[i];
            prm.precision = PMMM_F32;
            prm.n_max = 0;
            rc = pmmm_plan_create(&prm, stream, &c.plan);
            if (rc != PMMM_OK) break;
            b->cls.push_back(c);
        }
        b->cls[k].members.push_back(i);
    }
    for (auto &c : b->cls) {
        if (rc != PMMM_OK) break;
        rc = batch_alloc_class(c, s);
    }
    if (rc == PMMM_OK) {
        e = hipMalloc(&b->flag, sizeof(int));
        if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, sizeof(int), s);
        if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_prange, sizeof(int64_t) * 2 * nsys);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "batch workspace");
    }
    if (rc == PMMM_OK && b->cls.size() > 1) {
        const int nl = (int)b->cls.size() < kBatchStreams ? (int)b->cls.size() : kBatchStreams;
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (int k = 0; k < nl && e == hipSuccess; ++k) {
            hipStream_t st = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e == hipSuccess) b->side.push_back(st);
            hipEvent_t ev = nullptr;
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) b->join.push_back(ev);
        }
        if (e != hipSuccess) rc = hip_fail(e, "batch streams");
    }
    if (rc != PMMM_OK) {
        batch_destroy(b);
        return rc;
    }
    *out = b;
    return PMMM_OK;
}

void pmmm_batch_destroy(pmmm_batch batch) { batch_destroy(batch); }

int pmmm_batch_far_f32(pmmm_batch batch, const int64_t *offsets, const float *x, const float *y,
                       const float *z, const float *q, float *phi, float *gx, float *gy,
                       float *gz, void *stream) {
    return batch_far(batch, offsets, x, y, z, q, phi, gx, gy, gz, stream);
}

int pmmm_batch_classes(pmmm_batch batch) { return batch ? (int)batch->cls.size() : 0; }

int pmmm_batch_set_graphs(pmmm_batch batch, int enable) {
    if (!batch) {
        set_error("batch is NULL");
        return PMMM_EINVAL;
    }
    PMMM_HIP(hipDeviceSynchronize());
    drop_graph(batch);
    batch->use_graph = enable != 0;
    return PMMM_OK;
}

int pmmm_batch_sync_status(pmmm_batch batch) {
    if (!batch) {
        set_error("batch is NULL");
        return PMMM_EINVAL;
    }
    PMMM_HIP(hipStreamSynchronize(batch->last_stream));
    int flag = 0;
    PMMM_HIP(hipMemcpy(&flag, batch->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        const int zero = 0;
        PMMM_HIP(hipMemcpy(batch->flag, &zero, sizeof(int), hipMemcpyHostToDevice));
        set_error("open boundary: a particle lay outside [0, b)^3");
        return PMMM_EDOMAIN;
    }
    return PMMM_OK;
}

int pmmm_plan_autotune(pmmm_plan plan, int64_t n, const void *x, const void *y, const void *z,
                       const void *q, void *phi, void *gx, void *gy, void *gz, void *stream) {
    if (!plan) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (plan->tsize == sizeof(double))
        return autotune_impl<double>(plan, n, (const double *)x, (const double *)y,
                                     (const double *)z, (const double *)q, (double *)phi,
                                     (double *)gx, (double *)gy, (double *)gz, s);
    return autotune_impl<float>(plan, n, (const float *)x, (const float *)y, (const float *)z,
                                (const float *)q, (float *)phi, (float *)gx, (float *)gy,
                                (float *)gz, s);
}

int pmmm_plan_get_tuning(pmmm_plan plan, pmmm_tuning *out) {
    if (!plan || !out) {
        set_error("plan or out is NULL");
        return PMMM_EINVAL;
    }
    out->column_kernel = plan->tune_col_kernel;
    out->column_width = plan->tune_col_w;
    out->p2m_lanes = plan->tune_group;
    return PMMM_OK;
}

int pmmm_plan_set_tuning(pmmm_plan plan, const pmmm_tuning *in) {
    if (!plan || !in) {
        set_error("plan or in is NULL");
        return PMMM_EINVAL;
    }
    const int kind = in->column_kernel;
    if (kind != 0 && !column_kernel_fits(kind, plan->p, plan->nf, plan->tsize)) {
        set_error("column kernel form unknown or not fitting this plan");
        return PMMM_EINVAL;
    }
    if (in->column_width != 0) {
        int wmax = 0, rs = 0;
        const int w = in->column_width;
        if (kind != PMMM_COLUMN_TILE || w < 0 || (w & (w - 1)) != 0 ||
            column_shape(plan->p, plan->nf, plan->tsize, &wmax, &rs) == 0 || w > wmax) {
            set_error("column width needs the tile form and a power of two that fits LDS");
            return PMMM_EINVAL;
        }
    }
    const int g = in->p2m_lanes;
    if (g != 0 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64) {
        set_error("p2m_lanes must be 0, 4, 8, 16, 32 or 64");
        return PMMM_EINVAL;
    }
    plan->tune_col_kernel = kind;
    plan->tune_col_w = in->column_width;
    plan->tune_group = g;
    return PMMM_OK;
}

int pmmm_plan_sync_status(pmmm_plan plan) {
    if (!plan) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    PMMM_HIP(hipStreamSynchronize(plan->last_stream));
    int flag = 0;
    PMMM_HIP(hipMemcpy(&flag, plan->small + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        const int zero = 0;
        PMMM_HIP(hipMemcpy(plan->small + 1, &zero, sizeof(int), hipMemcpyHostToDevice));
        set_error("open boundary: a particle lay outside [0, b)^3");
        return PMMM_EDOMAIN;
    }
    return PMMM_OK;
}

size_t pmmm_plan_mesh_bytes(pmmm_plan plan, int which) {
    if (!plan) return 0;
    switch (which) {
        case PMMM_MESH_M:
        case PMMM_MESH_L:
            return (size_t)plan->P * plan->K * plan->tsize;
        case PMMM_MESH_GREEN:
            return (size_t)plan->ngreen * plan->tsize;
        default:
            return 0;
    }
}

int pmmm_plan_copy_mesh(pmmm_plan plan, int which, void *host_dst, size_t bytes) {
    if (!plan || !host_dst) {
        set_error("NULL plan or destination");
        return PMMM_EINVAL;
    }
    const size_t need = pmmm_plan_mesh_bytes(plan, which);
    if (need == 0 || bytes != need) {
        set_error("unknown mesh or wrong byte count");
        return PMMM_EINVAL;
    }
    const void *src = which == PMMM_MESH_M ? plan->M : (which == PMMM_MESH_L ? plan->L : plan->green);
    PMMM_HIP(hipStreamSynchronize(plan->last_stream));
    PMMM_HIP(hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
    return PMMM_OK;
}

int pmmm_plan_set_graphs(pmmm_plan plan, int enable) {
    if (!plan) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    if (!enable) {
        if (plan->gexec) PMMM_HIP(hipDeviceSynchronize());
        drop_plan_graph(plan);
    }
    plan->use_graph = enable ? 1 : 0;
    return PMMM_OK;
}

int pmmm_plan_set_profiling(pmmm_plan plan, unsigned mask) {
    if (!plan) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    plan->prof_mask = mask & ((1u << PMMM_NSTAGES) - 1);
    return PMMM_OK;
}

int pmmm_plan_read_profile(pmmm_plan plan, double *ms, int64_t *count, int reset) {
    if (!plan) {
        set_error("plan is NULL");
        return PMMM_EINVAL;
    }
    for (int st = 0; st < PMMM_NSTAGES; ++st) {
        for (auto &pr : plan->ev_pending[st]) {
            PMMM_HIP(hipEventSynchronize(pr.second));
            float t = 0.f;
            PMMM_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
            plan->prof_ms[st] += t;
            plan->prof_cnt[st] += 1;
            plan->ev_pool.push_back(pr.first);
            plan->ev_pool.push_back(pr.second);
        }
        plan->ev_pending[st].clear();
        if (ms) ms[st] = plan->prof_ms[st];
        if (count) count[st] = plan->prof_cnt[st];
        if (reset) {
            plan->prof_ms[st] = 0;
            plan->prof_cnt[st] = 0;
        }
    }
    return PMMM_OK;
}

const char *pmmm_error_string(int code) {
    switch (code) {
        case PMMM_OK: return "PMMM_OK";
        case PMMM_EINVAL: return "PMMM_EINVAL: invalid argument";
        case PMMM_ENOMEM: return "PMMM_ENOMEM: device allocation failed";
        case PMMM_EHIP: return "PMMM_EHIP: HIP runtime error";
        case PMMM_EDOMAIN: return "PMMM_EDOMAIN: particle outside the open-boundary box";
        case PMMM_EUNSUPPORTED: return "PMMM_EUNSUPPORTED: configuration not built";
        default: return "unknown PMMM error code";
    }
}

const char *pmmm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
