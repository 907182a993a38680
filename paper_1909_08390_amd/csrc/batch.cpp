// Host side of the batched 1D passes: many independent shock tubes of
// uneven size, adiabatic index (through K, Sec. II), tau and dt advanced
// together by the IMEX-SSP3(4,3,3) step of Sec. III.  Two execution modes:
//  - per-pass launches: one launch per fused pass covers every tile of
//    every tube (per-tube pass arguments and a tile table in device memory);
//  - persistent: one launch covers several whole steps; each work-group
//    owns a bin of items (tubes, or chunks of long outflow tubes stepped
//    over a region extended by 15 cells per step, temporal blocking) and
//    separates the passes with work-group barriers only.
// The autotuner times every plan (mode, tile width, tile order, chunk
// size, steps per launch, work-groups) on the caller's state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "imexlb.h"

using namespace imexlb;

namespace {

// One execution plan.  mode 0: per-pass launches with tiles of `tile`
// cells in `order` (0 tube by tube, 1 longest tubes first).  mode 1:
// persistent launches of up to `steps` steps; outflow tubes longer than
// `chunk` cells are split into chunks whose extended regions hold at most
// `chunk` cells; items go to `bins` work-groups of tile / 4 threads,
// longest items first to the least-loaded bin.
struct BatchPlan {
    int mode, tile, order, chunk, steps, bins;
};

constexpr BatchPlan kPlans[] = {
    {0, 256, 0, 0, 0, 0}, {0, 256, 1, 0, 0, 0}, {0, 512, 0, 0, 0, 0},
    {0, 512, 1, 0, 0, 0}, {0, 1024, 0, 0, 0, 0}, {0, 1024, 1, 0, 0, 0},
    {1, 1024, 1, 1024, 4, 512}, {1, 1024, 1, 1024, 4, 1024}, {1, 1024, 1, 1024, 8, 512},
    {1, 1024, 1, 1024, 8, 1024}, {1, 1024, 1, 2048, 4, 512}, {1, 1024, 1, 2048, 4, 1024},
    {1, 1024, 1, 2048, 8, 512}, {1, 1024, 1, 2048, 8, 1024}, {1, 512, 1, 512, 4, 1024},
    {1, 512, 1, 1024, 4, 1024}, {1, 512, 1, 1024, 8, 1024}, {1, 1024, 1, 4096, 4, 512},
    {1, 1024, 1, 4096, 4, 1024}, {1, 1024, 1, 4096, 8, 512}, {1, 1024, 1, 4096, 8, 1024},
};
constexpr int kNumPlans = (int)(sizeof(kPlans) / sizeof(kPlans[0]));
constexpr int kDefaultPlan = 2;     // per-pass launches, 512-cell tiles, tube order
constexpr int kMaxPersistBins = 1024;
constexpr int kCellsPerStep = 15;   // region growth per step: 3 passes x 5 cells

}  // namespace

struct imexlb_batch {
    int count = 0;
    int q[2] = {0, 0};
    int storage = IMEXLB_F64;
    int qm = 8;
    int nplanes = 0;
    size_t elem = 8;
    hipStream_t stream = nullptr;
    std::vector<imexlb_tube> tubes;
    std::vector<long long> soff, coff;  // state element offset, cell offset per tube
    long long state_elems = 0, ctot = 0;
    long long max_tiles = 0;            // tiles at the smallest width
    double p[2][kQMax] = {}, w[2][kQMax] = {};
    DevTables* d_tab = nullptr;
    StageArgs* d_args = nullptr;        // [3][count]: passes 3, 4, 5
    int* d_tiles = nullptr;             // (tube, first cell) per tile
    int tile = 512, order = 0, ntiles = 0;
    int plan = kDefaultPlan;
    // persistent mode: items, their pass arguments and bins of the current
    // plan; the private areas follow the five buffers in the workspace
    std::vector<PersistItem> items;
    std::vector<long long> item_priv;   // byte offset of each item's private area
    long long max_items = 0, priv_bytes = 0;
    PersistItem* d_items = nullptr;
    StageArgs* d_iargs = nullptr;       // [item][3]
    int* d_bin_start = nullptr;         // nbins + 1
    int* d_bin_items = nullptr;
    int nbins = 0;
    void* d_state = nullptr;
    void* d_work = nullptr;
    bool have_state = false;
    std::string err;
};

namespace {

constexpr int kTileAlign = 64;  // tube plane-sets start at multiples of 64 elements

imexlb_status bfail(imexlb_batch* b, imexlb_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

imexlb_status bhip(imexlb_batch* b, hipError_t e, const char* what) {
    return bfail(b, IMEXLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

char* state_ptr(const imexlb_batch* b, void* base, int i) {
    return (char*)base + (size_t)b->soff[i] * b->elem;
}

// Workspace: G3 | G4 | M^n | M3 | M4 (moments: 3 fields of ctot cells).
void* work_g(const imexlb_batch* b, int i) {
    return (char*)b->d_work + (size_t)i * align256((size_t)b->state_elems * b->elem);
}
double* work_m(const imexlb_batch* b, int i) {
    const size_t off = 2 * align256((size_t)b->state_elems * b->elem) +
                       (size_t)i * align256(3 * (size_t)b->ctot * sizeof(double));
    return (double*)((char*)b->d_work + off);
}

bool valid_tile(int t) {
    for (int k : kBatchTiles)
        if (k == t) return true;
    return false;
}

// Items of a persistent plan: (tube, region, own cells).  An outflow tube
// longer than `chunk` cells is split into n chunks of equal own length,
// each stepped over its cells extended by kCellsPerStep cells per step on
// each side that has a neighbour, with n the smallest count whose regions
// stay within `chunk` cells (so that a region fills whole tiles when chunk
// is a multiple of the tile width).
std::vector<PersistItem> make_items(const imexlb_batch* b, int chunk, int steps) {
    std::vector<PersistItem> out;
    const int ext = kCellsPerStep * steps;
    const int own_max = std::max(1, chunk - 2 * ext);
    for (int i = 0; i < b->count; ++i) {
        const imexlb_tube& t = b->tubes[i];
        const int n = (t.bc == IMEXLB_PERIODIC || t.nx <= chunk) ? 1 : (t.nx + own_max - 1) / own_max;
        for (int j = 0; j < n; ++j) {
            PersistItem m;
            std::memset(&m, 0, sizeof(m));
            m.soff = b->soff[i];
            m.coff = b->coff[i];
            m.nx = t.nx;
            m.own0 = (int)((long long)j * t.nx / n);
            m.own1 = (int)((long long)(j + 1) * t.nx / n);
            m.r0 = n == 1 ? 0 : std::max(0, m.own0 - ext);
            const int r1 = n == 1 ? t.nx : std::min(t.nx, m.own1 + ext);
            m.len = r1 - m.r0;
            m.pad = i;  // tube index (host only)
            out.push_back(m);
        }
    }
    return out;
}

// Private area of an item: F | G3 | G4 (planes x stride, storage type) and
// M^n | M3 | M4 (3 fields x stride, FP64); stride = region rounded up to 64.
long long item_stride(int len) { return (len + 63) / 64 * 64; }
size_t item_bytes(const imexlb_batch* b, int len) {
    const size_t st = (size_t)item_stride(len);
    return 3 * align256((size_t)b->nplanes * st * b->elem) + 3 * align256(3 * st * sizeof(double));
}

size_t private_bytes(const imexlb_batch* b, const std::vector<PersistItem>& items) {
    size_t t = 0;
    for (const PersistItem& m : items) t += item_bytes(b, m.len);
    return t;
}

size_t base_work_bytes(const imexlb_batch* b) {
    return 2 * align256((size_t)b->state_elems * b->elem) + 3 * align256(3 * (size_t)b->ctot * sizeof(double));
}

hipError_t upload_tiles(imexlb_batch* b) {
    std::vector<int> idx(b->count);
    for (int i = 0; i < b->count; ++i) idx[i] = i;
    if (b->order == 1)
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int x, int y) { return b->tubes[x].nx > b->tubes[y].nx; });
    std::vector<int> t;
    t.reserve(2 * b->max_tiles);
    for (int i : idx)
        for (int x0 = 0; x0 < b->tubes[i].nx; x0 += b->tile) {
            t.push_back(i);
            t.push_back(x0);
        }
    b->ntiles = (int)(t.size() / 2);
    hipError_t e = hipMemcpyAsync(b->d_tiles, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

hipError_t upload_args(imexlb_batch* b) {
    std::vector<StageArgs> args(3 * (size_t)b->count);
    for (int i = 0; i < b->count; ++i) {
        const imexlb_tube& tb = b->tubes[i];
        StageArgs a;
        std::memset(&a, 0, sizeof(a));
        a.tab = b->d_tab;
        a.nx = tb.nx;
        a.ny = 1;
        a.bcx = tb.bc;
        a.ntx = (tb.nx + b->tile - 1) / b->tile;
        a.nty = 1;
        a.qm = b->qm;
        a.plane_stride = tb.nx;
        a.mstride = b->ctot;
        a.inv_dx = tb.nx / tb.lx;
        stage_coefficients(tb.dt, tb.tau, a);
        a.chi_fac = (double)(tb.K + kDTotal - 1);
        a.dk = (double)(kDTotal + tb.K);
        StageArgs pa[3];
        pass_args(a, state_ptr(b, b->d_state, i), state_ptr(b, work_g(b, 0), i), state_ptr(b, work_g(b, 1), i),
                  work_m(b, 0) + b->coff[i], work_m(b, 1) + b->coff[i], work_m(b, 2) + b->coff[i], pa);
        for (int k = 0; k < 3; ++k) args[(size_t)k * b->count + i] = pa[k];
    }
    hipError_t e = hipMemcpyAsync(b->d_args, args.data(), args.size() * sizeof(StageArgs),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

// Items, private areas, pass arguments and bins of the current persistent
// plan (needs the bound workspace).
hipError_t upload_persist(imexlb_batch* b) {
    const BatchPlan& pl = kPlans[b->plan];
    b->items = make_items(b, pl.chunk, pl.steps);
    const int ni = (int)b->items.size();
    b->item_priv.assign(ni, 0);
    char* base = (char*)b->d_work + base_work_bytes(b);
    size_t off = 0;
    std::vector<StageArgs> args(3 * (size_t)ni);
    for (int k = 0; k < ni; ++k) {
        const PersistItem& m = b->items[k];
        const imexlb_tube& tb = b->tubes[m.pad];
        b->item_priv[k] = (long long)off;
        const size_t st = (size_t)item_stride(m.len);
        const size_t pf = align256((size_t)b->nplanes * st * b->elem), pm = align256(3 * st * sizeof(double));
        char* p = base + off;
        off += item_bytes(b, m.len);
        StageArgs a;
        std::memset(&a, 0, sizeof(a));
        a.tab = b->d_tab;
        a.nx = m.len;
        a.ny = 1;
        a.bcx = tb.bc;
        a.ntx = (m.len + pl.tile - 1) / pl.tile;
        a.nty = 1;
        a.qm = b->qm;
        a.plane_stride = (long long)st;
        a.mstride = (long long)st;
        a.inv_dx = tb.nx / tb.lx;
        stage_coefficients(tb.dt, tb.tau, a);
        a.chi_fac = (double)(tb.K + kDTotal - 1);
        a.dk = (double)(kDTotal + tb.K);
        StageArgs pa[3];
        pass_args(a, p, p + pf, p + 2 * pf, (double*)(p + 3 * pf), (double*)(p + 3 * pf + pm),
                  (double*)(p + 3 * pf + 2 * pm), pa);
        for (int q = 0; q < 3; ++q) args[3 * (size_t)k + q] = pa[q];
    }
    // longest items first, each to the least-loaded bin
    const int nb = std::min(pl.bins, ni);
    std::vector<int> idx(ni);
    for (int k = 0; k < ni; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return b->items[x].len > b->items[y].len; });
    std::vector<long long> load(nb, 0);
    std::vector<std::vector<int>> bins(nb);
    for (int k : idx) {
        int best = 0;
        for (int q = 1; q < nb; ++q)
            if (load[q] < load[best]) best = q;
        bins[best].push_back(k);
        load[best] += b->items[k].len;
    }
    std::vector<int> start(nb + 1, 0), flat;
    flat.reserve(ni);
    for (int q = 0; q < nb; ++q) {
        start[q] = (int)flat.size();
        flat.insert(flat.end(), bins[q].begin(), bins[q].end());
    }
    start[nb] = (int)flat.size();
    b->nbins = nb;
    hipError_t e = hipMemcpyAsync(b->d_items, b->items.data(), ni * sizeof(PersistItem), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_iargs, args.data(), args.size() * sizeof(StageArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_bin_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_bin_items, flat.data(), flat.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

// Device tables of the current plan (tile table or persistent items).
hipError_t apply_plan(imexlb_batch* b) {
    const BatchPlan& pl = kPlans[b->plan];
    b->tile = pl.tile;
    b->order = pl.order;
    if (pl.mode == 0) return upload_tiles(b);
    return b->d_work ? upload_persist(b) : hipSuccess;
}

hipError_t recompute_moments(imexlb_batch* b) {
    const bool f32 = b->storage == IMEXLB_F32;
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->count && e == hipSuccess; ++i)
        e = launch_moments(1, f32, b->d_tab, state_ptr(b, b->d_state, i), work_m(b, 0) + b->coff[i],
                           b->tubes[i].nx, b->ctot, (double)(kDTotal + b->tubes[i].K), b->stream);
    return e;
}

// Persistent mode: launches of up to `steps` steps, reading the state and
// moments from one buffer pair and writing the other (the bound state and
// M^n, or the G3 and M3 workspace slots).  With an odd number of launches
// the state is first copied to the second pair, so that the last launch
// writes the bound state.  With ev, ev[0] and ev[1] bracket all launches.
hipError_t run_persist(imexlb_batch* b, int nsteps, hipEvent_t* ev) {
    const BatchPlan& pl = kPlans[b->plan];
    const int nl = (nsteps + pl.steps - 1) / pl.steps;
    void* fb[2] = {b->d_state, work_g(b, 0)};
    double* mb[2] = {work_m(b, 0), work_m(b, 1)};
    const size_t sb = (size_t)b->state_elems * b->elem, mbytes = 3 * (size_t)b->ctot * sizeof(double);
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[0], b->stream);
    int cur = 0;
    if (nl % 2 == 1 && e == hipSuccess) {
        e = hipMemcpyAsync(fb[1], fb[0], sb, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(mb[1], mb[0], mbytes, hipMemcpyDeviceToDevice, b->stream);
        cur = 1;
    }
    for (int l = 0; l < nl && e == hipSuccess; ++l) {
        PersistIO io;
        io.f_in = fb[cur];
        io.f_out = fb[1 - cur];
        io.m_in = mb[cur];
        io.m_out = mb[1 - cur];
        io.ctot = b->ctot;
        io.nplanes = b->nplanes;
        const int ns = std::min(pl.steps, nsteps - l * pl.steps);
        e = launch_stage1d_persist(b->storage == IMEXLB_F32, b->qm, pl.tile, b->d_iargs, b->d_items, b->d_bin_start,
                                   b->d_bin_items, b->nbins, io, ns, b->stream);
        cur = 1 - cur;
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], b->stream);
    return e;
}

hipError_t run(imexlb_batch* b, int nsteps, hipEvent_t* ev) {
    if (kPlans[b->plan].mode == 1) return run_persist(b, nsteps, ev);
    const bool f32 = b->storage == IMEXLB_F32;
    const int kinds[3] = {kStage3, kStage4, kStage5};
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[0], b->stream);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s)
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            e = launch_stage1d_batch(f32, kinds[k], b->qm, b->tile, b->d_args + (size_t)k * b->count,
                                     (const int2*)b->d_tiles, b->ntiles, b->stream);
            if (e == hipSuccess && ev) e = hipEventRecord(ev[3 * s + k + 1], b->stream);
        }
    return e;
}

}  // namespace

extern "C" {

imexlb_status imexlb_batch_create(const imexlb_tube* tubes, int count, int q_phi, int q_chi, int storage,
                                  void* hip_stream, imexlb_batch** out) {
    if (!out) return IMEXLB_EINVAL;
    *out = nullptr;
    auto bad = [](const std::string& m) {
        std::fprintf(stderr, "imexlb_batch_create: %s\n", m.c_str());
        return IMEXLB_EINVAL;
    };
    if (!tubes || count < 1) return bad("need at least one tube");
    if (q_phi < 3 || q_phi > kQMax) return bad("q_phi must be in [3, 16]");
    if (q_chi < 1 || q_chi > kQMax) return bad("q_chi must be in [1, 16]");
    if (storage != IMEXLB_F64 && storage != IMEXLB_F32) return bad("bad storage");
    imexlb_batch* b = new (std::nothrow) imexlb_batch();
    if (!b) return IMEXLB_ENOMEM;
    b->count = count;
    b->q[0] = q_phi;
    b->q[1] = q_chi;
    b->storage = storage;
    b->elem = storage == IMEXLB_F32 ? 4 : 8;
    b->qm = (q_phi <= 8 && q_chi <= 8) ? 8 : 16;
    b->nplanes = q_phi + q_chi;
    b->stream = (hipStream_t)hip_stream;
    for (int s = 0; s < 2; ++s)
        if (!quadrature_rule(b->q[s], b->p[s], b->w[s])) {
            delete b;
            return bad("quadrature");
        }
    double pmax = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < b->q[s]; ++k) pmax = std::fmax(pmax, std::fabs(b->p[s][k]));
    b->tubes.assign(tubes, tubes + count);
    b->soff.resize(count);
    b->coff.resize(count);
    long long so = 0, co = 0, mt = 0;
    for (int i = 0; i < count; ++i) {
        const imexlb_tube& t = tubes[i];
        std::string why;
        if (t.nx < 1) why = "nx must be >= 1";
        else if (!(t.lx > 0.0)) why = "length must be > 0";
        else if (t.K < 0) why = "K must be >= 0";
        else if (!(t.tau > 0.0) || !std::isfinite(t.tau)) why = "tau must be > 0";
        else if (!(t.dt > 0.0) || !std::isfinite(t.dt)) why = "dt must be > 0";
        else if (t.bc != IMEXLB_OUTFLOW && t.bc != IMEXLB_PERIODIC) why = "bad bc";
        else if (pmax * t.dt * t.nx / t.lx > 1.0) why = "CFL > 1";
        else if (((long long)t.nx + 1024) * (long long)b->elem >= (1LL << 31)) why = "tube too long";
        if (!why.empty()) {
            delete b;
            return bad("tube " + std::to_string(i) + ": " + why);
        }
        b->soff[i] = so;
        b->coff[i] = co;
        const long long el = (long long)b->nplanes * t.nx;
        so += (el + kTileAlign - 1) / kTileAlign * kTileAlign;
        co += t.nx;
        mt += (t.nx + kBatchTiles[0] - 1) / kBatchTiles[0];
    }
    b->state_elems = so;
    b->ctot = co;
    b->max_tiles = mt;
    if (b->ctot >= (1LL << 31)) {
        delete b;
        return bad("too many cells");
    }
    // the largest item list and private area over the persistent plans
    for (const BatchPlan& pl : kPlans) {
        if (pl.mode != 1) continue;
        const std::vector<PersistItem> it = make_items(b, pl.chunk, pl.steps);
        b->max_items = std::max(b->max_items, (long long)it.size());
        b->priv_bytes = std::max(b->priv_bytes, (long long)private_bytes(b, it));
    }
    hipError_t e = upload_tables(1, b->q, b->p, b->w, 0, &b->d_tab, b->stream);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_args, 3 * (size_t)count * sizeof(StageArgs));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_tiles, 2 * (size_t)mt * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_items, (size_t)b->max_items * sizeof(PersistItem));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_iargs, 3 * (size_t)b->max_items * sizeof(StageArgs));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_bin_start, (kMaxPersistBins + 1) * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_bin_items, (size_t)b->max_items * sizeof(int));
    if (e == hipSuccess) e = apply_plan(b);
    if (e != hipSuccess) {
        std::fprintf(stderr, "imexlb_batch_create: %s\n", hipGetErrorString(e));
        imexlb_batch_destroy(b);
        return e == hipErrorOutOfMemory ? IMEXLB_ENOMEM : IMEXLB_EHIP;
    }
    *out = b;
    return IMEXLB_OK;
}

void imexlb_batch_destroy(imexlb_batch* b) {
    if (!b) return;
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->d_args) (void)hipFree(b->d_args);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_iargs) (void)hipFree(b->d_iargs);
    if (b->d_bin_start) (void)hipFree(b->d_bin_start);
    if (b->d_bin_items) (void)hipFree(b->d_bin_items);
    delete b;
}

imexlb_status imexlb_batch_set_stream(imexlb_batch* b, void* s) {
    if (!b) return IMEXLB_EINVAL;
    b->stream = (hipStream_t)s;
    return IMEXLB_OK;
}

size_t imexlb_batch_state_bytes(const imexlb_batch* b) {
    return b ? (size_t)b->state_elems * b->elem : 0;
}

size_t imexlb_batch_workspace_bytes(const imexlb_batch* b) {
    if (!b) return 0;
    return base_work_bytes(b) + (size_t)b->priv_bytes;
}

long long imexlb_batch_cells(const imexlb_batch* b) { return b ? b->ctot : 0; }

imexlb_status imexlb_batch_layout(const imexlb_batch* b, long long* so, long long* co) {
    if (!b) return IMEXLB_EINVAL;
    for (int i = 0; i < b->count; ++i) {
        if (so) so[i] = b->soff[i];
        if (co) co[i] = b->coff[i];
    }
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_bind(imexlb_batch* b, void* d_state, void* d_work) {
    if (!b) return IMEXLB_EINVAL;
    if (!d_state || !d_work) return bfail(b, IMEXLB_EINVAL, "bind: NULL buffer");
    if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
        return bfail(b, IMEXLB_EINVAL, "bind: buffers must be 256-byte aligned");
    b->d_state = d_state;
    b->d_work = d_work;
    b->have_state = false;
    hipError_t e = upload_args(b);
    if (e == hipSuccess && kPlans[b->plan].mode == 1) e = upload_persist(b);
    if (e != hipSuccess) return bhip(b, e, "bind");
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_set_equilibrium(imexlb_batch* b, const double* n, const double* u, const double* T) {
    if (!b) return IMEXLB_EINVAL;
    if (!b->d_state) return bfail(b, IMEXLB_ESTATE, "set_equilibrium: not bound");
    if (!n || !u || !T) return bfail(b, IMEXLB_EINVAL, "set_equilibrium: NULL field");
    const bool f32 = b->storage == IMEXLB_F32;
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->count && e == hipSuccess; ++i) {
        const long long c = b->coff[i];
        e = launch_init_equilibrium(1, f32, b->d_tab, n + c, u + c, nullptr, T + c, state_ptr(b, b->d_state, i),
                                    nullptr, b->tubes[i].nx, (double)(b->tubes[i].K + kDTotal - 1), b->stream);
    }
    if (e == hipSuccess) e = recompute_moments(b);
    if (e != hipSuccess) return bhip(b, e, "set_equilibrium");
    b->have_state = true;
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_state_changed(imexlb_batch* b) {
    if (!b) return IMEXLB_EINVAL;
    if (!b->d_state) return bfail(b, IMEXLB_ESTATE, "state_changed: not bound");
    hipError_t e = recompute_moments(b);
    if (e != hipSuccess) return bhip(b, e, "state_changed");
    b->have_state = true;
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_step(imexlb_batch* b, int nsteps) {
    if (!b) return IMEXLB_EINVAL;
    if (nsteps < 0) return bfail(b, IMEXLB_EINVAL, "step: nsteps < 0");
    if (!b->have_state) return bfail(b, IMEXLB_ESTATE, "step: no state");
    hipError_t e = run(b, nsteps, nullptr);
    if (e != hipSuccess) return bhip(b, e, "step");
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_step_timed(imexlb_batch* b, int nsteps, double ms[3]) {
    if (!b || !ms) return IMEXLB_EINVAL;
    if (nsteps < 0) return bfail(b, IMEXLB_EINVAL, "step_timed: nsteps < 0");
    if (!b->have_state) return bfail(b, IMEXLB_ESTATE, "step_timed: no state");
    const bool persist = kPlans[b->plan].mode == 1;
    const int ne = persist ? 2 : 3 * nsteps + 1;
    std::vector<hipEvent_t> ev(ne);
    int made = 0;
    hipError_t e = hipSuccess;
    for (; made < ne && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) --made;
    if (e == hipSuccess) e = run(b, nsteps, ev.data());
    if (e == hipSuccess) e = hipEventSynchronize(ev[ne - 1]);
    if (persist && e == hipSuccess && nsteps > 0) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, ev[0], ev[1]);
        ms[0] += t;
    }
    for (int s = 0; !persist && s < nsteps && e == hipSuccess; ++s)
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ev[3 * s + k], ev[3 * s + k + 1]);
            ms[k] += t;
        }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return bhip(b, e, "step_timed");
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_moments(const imexlb_batch* b, double* n, double* u, double* T) {
    if (!b) return IMEXLB_EINVAL;
    imexlb_batch* m = const_cast<imexlb_batch*>(b);
    if (!b->have_state) return bfail(m, IMEXLB_ESTATE, "moments: no state");
    double* dst[3] = {n, u, T};
    const double* M = work_m(b, 0);
    for (int f = 0; f < 3; ++f) {
        if (!dst[f]) continue;
        hipError_t e = hipMemcpyAsync(dst[f], M + (size_t)f * b->ctot, (size_t)b->ctot * sizeof(double),
                                      hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return bhip(m, e, "moments");
    }
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_set_tiling(imexlb_batch* b, int tile, int order) {
    if (!b) return IMEXLB_EINVAL;
    if (!valid_tile(tile) || (order != 0 && order != 1))
        return bfail(b, IMEXLB_EINVAL, "set_tiling: tile must be 256, 512 or 1024 and order 0 or 1");
    for (int i = 0; i < kNumPlans; ++i)
        if (kPlans[i].mode == 0 && kPlans[i].tile == tile && kPlans[i].order == order)
            return imexlb_batch_set_plan(b, i);
    return bfail(b, IMEXLB_EINVAL, "set_tiling: no such plan");
}

imexlb_status imexlb_batch_get_tiling(const imexlb_batch* b, int* tile, int* order) {
    if (!b) return IMEXLB_EINVAL;
    if (tile) *tile = b->tile;
    if (order) *order = b->order;
    return IMEXLB_OK;
}

int imexlb_batch_plan_count(void) { return kNumPlans; }

imexlb_status imexlb_batch_plan_info(int plan, int info[6]) {
    if (plan < 0 || plan >= kNumPlans || !info) return IMEXLB_EINVAL;
    const BatchPlan& p = kPlans[plan];
    info[0] = p.mode;
    info[1] = p.tile;
    info[2] = p.order;
    info[3] = p.chunk;
    info[4] = p.steps;
    info[5] = p.bins;
    return IMEXLB_OK;
}

imexlb_status imexlb_batch_set_plan(imexlb_batch* b, int plan) {
    if (!b) return IMEXLB_EINVAL;
    if (plan < 0 || plan >= kNumPlans) return bfail(b, IMEXLB_EINVAL, "set_plan: no such plan");
    b->plan = plan;
    hipError_t e = apply_plan(b);
    if (e != hipSuccess) return bhip(b, e, "set_plan");
    return IMEXLB_OK;
}

int imexlb_batch_get_plan(const imexlb_batch* b) { return b ? b->plan : -1; }

imexlb_status imexlb_batch_tune(imexlb_batch* b, int nsteps, double* ms_out) {
    if (!b) return IMEXLB_EINVAL;
    if (nsteps < 1) return bfail(b, IMEXLB_EINVAL, "tune: nsteps < 1");
    if (!b->have_state) return bfail(b, IMEXLB_ESTATE, "tune: no state");
    const size_t sb = imexlb_batch_state_bytes(b);
    const size_t mb = 3 * (size_t)b->ctot * sizeof(double);
    char* save = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&save, sb + mb);
    if (e == hipSuccess) e = hipMemcpyAsync(save, b->d_state, sb, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(save + sb, work_m(b, 0), mb, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto restore = [&]() {
        hipError_t r = hipMemcpyAsync(b->d_state, save, sb, hipMemcpyDeviceToDevice, b->stream);
        if (r == hipSuccess) r = hipMemcpyAsync(work_m(b, 0), save + sb, mb, hipMemcpyDeviceToDevice, b->stream);
        return r;
    };
    double best = 1e300;
    int best_plan = b->plan;
    for (int ci = 0; ci < kNumPlans && e == hipSuccess; ++ci) {
        b->plan = ci;
        e = apply_plan(b);
        if (e == hipSuccess) e = run(b, 1, nullptr);  // untimed first step
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = run(b, nsteps, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = restore();
        const double per = (double)ms / nsteps;
        if (ms_out) ms_out[ci] = per;
        if (e == hipSuccess && per < best) {
            best = per;
            best_plan = ci;
        }
    }
    b->plan = best_plan;
    if (e == hipSuccess) e = apply_plan(b);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (save) (void)hipFree(save);
    if (e != hipSuccess) return bhip(b, e, "tune");
    return IMEXLB_OK;
}

const char* imexlb_batch_last_error(const imexlb_batch* b) { return b ? b->err.c_str() : "NULL batch"; }

}  // extern "C"
