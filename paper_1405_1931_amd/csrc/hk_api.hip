// C-ABI of the library: argument checks, brick choice, workspace cache and
// launches.  See include/hk.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/hk.h"
#include "hk_launch.h"

namespace hk {
namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kErrBytes = 256;

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int ceil_pow2(int v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

// ceil(log2(v)) for 1 <= v <= INT32_MAX (31 at most: 1 << 31 is not an int)
int log2i(int v) {
    int l = 0;
    while (l < 31 && (1 << l) < v) ++l;
    return l;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------- bricks

std::mutex g_brick_mu;
int g_force_by = 0, g_force_bz = 0;
std::map<uint32_t, std::pair<int, int>> g_tuned;  // bucket -> (by, bz)

uint32_t bucket_of(int nx, int ny, int nz) {
    return (uint32_t)(log2i(nx) | (log2i(ny) << 8) | (log2i(nz) << 16));
}

// ceil(a / b) without overflow for a up to INT32_MAX
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t n_bricks(int nx, int ny, int nz, int by, int bz) { return cdiv(nx, 64) * cdiv(ny, by) * cdiv(nz, bz); }

// Every brick costs a fixed latency, so bricks are as large as the lattice
// allows; a lone small lattice trades some of that for more bricks in flight
// (down to 64 x 8 x 8), while a lattice of a batch never does, since the
// batch itself fills the chip.
void heuristic_brick(int nx, int ny, int nz, bool batch, int *by, int *bz) {
    int y = std::min(16, ceil_pow2(ny)), z = std::min(16, ceil_pow2(nz));
    while (!batch && n_bricks(nx, ny, nz, y, z) < 1024 && y * z > 64) {
        if (y >= z) y >>= 1; else z >>= 1;
    }
    *by = y;
    *bz = z;
}

void choose_brick(int nx, int ny, int nz, bool batch, int *by, int *bz) {
    std::lock_guard<std::mutex> lk(g_brick_mu);
    if (g_force_by > 0) {
        *by = g_force_by;
        *bz = g_force_bz;
        return;
    }
    auto it = g_tuned.find(bucket_of(nx, ny, nz));
    if (it != g_tuned.end()) {
        *by = it->second.first;
        *bz = it->second.second;
        return;
    }
    heuristic_brick(nx, ny, nz, batch, by, bz);
}

// ---------------------------------------------------------------- plans

struct Layout {
    int64_t occ, root, wpre, face, bcount, npar, nkey, nsize, nlpos, nrootkey, runlab, icomp, icount, nrun,
        slab, rowo, rowcnt, blksum, total;
};

// multiplier and shift of fast_div for the divisor d (1 <= d < 2^31)
void magic_div(uint32_t d, uint32_t *m, int32_t *l) {
    if (d <= 1) {
        *m = 0;
        *l = 0;
        return;
    }
    int k = 0;
    while (((uint64_t)1 << k) < d) ++k;  // ceil(log2 d)
    *m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << k) - d)) / d + 1);
    *l = k;
}

// geometry (no pointers) of one lattice; false if it cannot be handled
bool make_geo(int nx, int ny, int nz, uint32_t mask, int by, int bz, Geo *g) {
    std::memset(g, 0, sizeof(*g));
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->mask = mask;
    g->BY = by;
    g->BZ = bz;
    g->lby = log2i(by);
    g->lbz = log2i(bz);
    g->R = by * bz;
    g->nbx = (int)cdiv(nx, 64);
    g->nby = (int)cdiv(ny, by);
    g->nbz = (int)cdiv(nz, bz);
    const int64_t nb = (int64_t)g->nbx * g->nby * g->nbz;
    const int exm = std::min(64, nx);
    const int64_t c1 = 2 * ((g->R + 1) / 2) + 2 * ((exm * bz + 1) / 2) + 2 * ((exm * by + 1) / 2);
    const int64_t c2 = ((int64_t)exm * g->R + 1) / 2;
    const int64_t cap = std::max<int64_t>(1, std::min(c1, c2));
    if (nb > INT32_MAX || nb * cap > INT32_MAX || nb * g->R > ((int64_t)1 << 40)) return false;
    g->nb = (int)nb;
    g->cap = (int)cap;
    // a row of exm sites holds <= ceil(exm/2) runs; a multiple of four keeps
    // every brick's run table 8-byte aligned for the relabel pass
    g->runcap = (g->R * ((exm + 1) / 2) + 3) & ~3;
    g->icap = (int)c2;                   // components of a brick <= half its sites
    if (nb * (int64_t)g->runcap > ((int64_t)1 << 40) || nb * (int64_t)g->icap > ((int64_t)1 << 40)) return false;
    g->fstride = 2 * g->R;
    g->rows = ny * nz;  // <= N <= INT32_MAX
    g->nblk = (int)(((int64_t)g->rows + WG - 1) / WG);
    magic_div((uint32_t)((int64_t)nx * ny), &g->dm_xy, &g->ds_xy);  // nx ny <= N < 2^31
    magic_div((uint32_t)nx, &g->dm_x, &g->ds_x);
    return true;
}

Layout layout_of(const Geo &g, int64_t base) {
    Layout L;
    int64_t o = base;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int64_t words = (int64_t)g.nb * g.R;
    const int64_t nodes = (int64_t)g.nb * g.cap;
    L.occ = take(words * 8);
    L.root = take(words * 8);
    L.wpre = take(words * 4);
    L.face = take((int64_t)g.nb * g.fstride * 2);
    L.bcount = take((int64_t)g.nb * 4);
    L.npar = take(nodes * 4);
    L.nkey = take(nodes * 4);
    L.nsize = take(nodes * 4);
    L.nlpos = take(nodes * 2);
    L.nrootkey = take(nodes * 4);
    L.runlab = take((int64_t)g.nb * g.runcap * 2);
    L.icomp = take((int64_t)g.nb * g.icap * 4);
    L.icount = take((int64_t)g.nb * 4);
    L.nrun = take((int64_t)g.nb * 4);
    L.slab = take(nodes * 4);
    L.rowo = take(words * 2);
    L.rowcnt = take((int64_t)g.rows * 4);
    L.blksum = take((int64_t)g.nblk * 4);
    L.total = o - base;
    return L;
}

void bind(Geo *g, char *base, const Layout &L) {
    g->occ = (uint64_t *)(base + L.occ);
    g->root = (uint64_t *)(base + L.root);
    g->wpre = (int32_t *)(base + L.wpre);
    g->face = (uint16_t *)(base + L.face);
    g->bcount = (int32_t *)(base + L.bcount);
    g->npar = (int32_t *)(base + L.npar);
    g->nkey = (int32_t *)(base + L.nkey);
    g->nsize = (int32_t *)(base + L.nsize);
    g->nlpos = (uint16_t *)(base + L.nlpos);
    g->nrootkey = (int32_t *)(base + L.nrootkey);
    g->runlab = (uint16_t *)(base + L.runlab);
    g->icomp = (uint32_t *)(base + L.icomp);
    g->icount = (int32_t *)(base + L.icount);
    g->nrun = (int32_t *)(base + L.nrun);
    g->slab = (int32_t *)(base + L.slab);
    g->rowo = (uint16_t *)(base + L.rowo);
    g->rowcnt = (int32_t *)(base + L.rowcnt);
    g->blksum = (int32_t *)(base + L.blksum);
}

// the fallback counters sit in the workspace's first block, after the
// check word (the block is cleared when the workspace is allocated)
constexpr int64_t kDbgOffset = 64;
static_assert(kDbgOffset + DBG_N * 4 <= kErrBytes, "the counters fit the first block");
uint32_t *dbg_counters(char *ws_base) { return (uint32_t *)(ws_base + kDbgOffset); }

int check_shape(int32_t nx, int32_t ny, int32_t nz, uint32_t mask) {
    if (nx < 1 || ny < 1 || nz < 1 || mask > 7u) return HK_ERR_INVALID_ARG;
    if ((int64_t)nx * ny * nz > INT32_MAX) return HK_ERR_TOO_LARGE;
    return HK_OK;
}

// plan one lattice: geometry with a brick that fits
int plan_lattice(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g, bool batch = false) {
    int by, bz;
    choose_brick(nx, ny, nz, batch, &by, &bz);
    if (make_geo(nx, ny, nz, mask, by, bz, g)) return HK_OK;
    // fall back to smaller bricks (fewer node slots per brick)
    for (int r = by * bz / 2; r >= 1; r /= 2) {
        const int y = std::min(by, r), z = std::max(1, r / std::min(by, r));
        if (make_geo(nx, ny, nz, mask, y, z, g)) return HK_OK;
    }
    return HK_ERR_TOO_LARGE;
}

// ---------------------------------------------------------------- workspace

struct Workspace {
    char *base = nullptr;
    int64_t bytes = 0;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// returns a workspace of at least `bytes` (plus the error word) for (device, stream)
int get_workspace(hipStream_t stream, int64_t bytes, Workspace **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    Workspace &ws = g_ws[{dev, stream}];
    const int64_t need = bytes + kErrBytes;
    if (ws.bytes < need) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return HK_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone) return HK_ERR_NO_WORKSPACE;
        if (ws.base) {
            if (hipStreamSynchronize(stream) != hipSuccess) return HK_ERR_HIP;
            (void)hipFree(ws.base);
            ws.base = nullptr;
            ws.bytes = 0;
        }
        const int64_t grow = align_up(need + need / 8);
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)grow) != hipSuccess) {
            (void)hipGetLastError();
            return HK_ERR_HIP;
        }
        if (hipMemset(p, 0, (size_t)kErrBytes) != hipSuccess) {
            (void)hipFree(p);
            return HK_ERR_HIP;
        }
        ws.base = (char *)p;
        ws.bytes = grow;
    }
    *out = &ws;
    return HK_OK;
}

}  // namespace

// accessors for the autotuner (hk_tune.hip); all take g_brick_mu
void brick_forced(int *by, int *bz) {
    std::lock_guard<std::mutex> lk(g_brick_mu);
    *by = g_force_by;
    *bz = g_force_bz;
}
void brick_force(int by, int bz) {
    std::lock_guard<std::mutex> lk(g_brick_mu);
    g_force_by = by;
    g_force_bz = bz;
}
std::vector<std::pair<uint32_t, std::pair<int, int>>> brick_table() {
    std::lock_guard<std::mutex> lk(g_brick_mu);
    return {g_tuned.begin(), g_tuned.end()};
}
void brick_table_set(uint32_t bucket, int by, int bz) {
    std::lock_guard<std::mutex> lk(g_brick_mu);
    g_tuned[bucket] = {by, bz};
}
uint32_t brick_bucket(int nx, int ny, int nz) { return bucket_of(nx, ny, nz); }


// exposed to the batched path
int plan_lattice_ext(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g) {
    return plan_lattice(nx, ny, nz, mask, g, true);
}
// a single lattice's plan, as hk_label makes it
int plan_lattice_one(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g) {
    return plan_lattice(nx, ny, nz, mask, g, false);
}
int64_t lattice_bytes(const Geo &g) { return layout_of(g, 0).total; }
void bind_lattice(Geo *g, char *base) { bind(g, base, layout_of(*g, 0)); }
uint32_t *workspace_dbg(int32_t *err) { return dbg_counters((char *)err); }
int acquire_workspace(hipStream_t st, int64_t bytes, char **base, int32_t **err) {
    Workspace *ws = nullptr;
    const int rc = get_workspace(st, bytes, &ws);
    if (rc != HK_OK) return rc;
    *err = (int32_t *)ws->base;
    *base = ws->base + kErrBytes;
    return HK_OK;
}
std::mutex &workspace_mutex() { return g_ws_mu; }

// ---------------------------------------------------------------- profiling
// While enabled, every hk_label call records kPhases + 1 events on its
// stream around its kernels; hk_profile_read folds them into per-phase sums.
namespace {
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::vector<hipEvent_t>> g_prof_calls;  // events of unread calls
std::vector<hipEvent_t> g_prof_pool;                 // recycled events
}  // namespace

hipEvent_t *profile_events() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return nullptr;
    std::vector<hipEvent_t> ev(kPhases + 1);
    for (auto &e : ev) {
        if (!g_prof_pool.empty()) {
            e = g_prof_pool.back();
            g_prof_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return nullptr;
        }
    }
    g_prof_calls.push_back(std::move(ev));
    return g_prof_calls.back().data();
}
int ensure_capture_arena();  // hk_batched.hip
void release_batched();       // hk_batched.hip

}  // namespace hk

using namespace hk;

extern "C" {

int64_t hk_max_clusters(int32_t nx, int32_t ny, int32_t nz) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    return ((int64_t)nx * ny * nz + 1) / 2;
}

int64_t hk_workspace_bytes(int32_t nx, int32_t ny, int32_t nz) {
    const int rc = check_shape(nx, ny, nz, 0);
    if (rc != HK_OK) return rc;
    Geo g;
    const int pr = plan_lattice(nx, ny, nz, 0, &g);
    if (pr != HK_OK) return pr;
    return layout_of(g, 0).total + kErrBytes;
}

}  // extern "C"

namespace {

// the droplet statistics requested with a labelling (hk_label_droplets)
struct DsArgs {
    int64_t min_size;
    double r_max;
    int32_t n_bins;
    int64_t *hist, *counts;
    double *sums;
};

// workspace bytes of the statistics' partial accumulators
int64_t ds_bytes(int n_bins) {
    return align_up((int64_t)DS_PARTS * (n_bins + 2) * 8) + align_up((int64_t)DS_PARTS * 3 * 8);
}

// hk_label, hk_label_pred and hk_label_droplets: one lattice, the field read
// by predicate pk, with the droplet statistics when ds is non-null
int label_one(const void *field, int pk, int32_t tkey, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
              int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream, const DsArgs *ds = nullptr) {
    if (!field || !labels || !n_clusters) return HK_ERR_INVALID_ARG;
    int rc = check_shape(nx, ny, nz, periodic_mask);
    if (rc != HK_OK) return rc;
    if ((const void *)labels == field) return HK_ERR_INVALID_ARG;
    Geo g;
    rc = plan_lattice(nx, ny, nz, periodic_mask, &g);
    if (rc != HK_OK) return rc;
    const Layout L = layout_of(g, 0);
    const int64_t lat = ds ? align_up(L.total) : L.total;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace *ws = nullptr;
    rc = get_workspace(stream, lat + (ds ? ds_bytes(ds->n_bins) : 0), &ws);
    if (rc != HK_OK) return rc;
    g.err = (int32_t *)ws->base;
    g.dbg = dbg_counters(ws->base);
    bind(&g, ws->base + kErrBytes, L);
    if (ds) {
        char *p = ws->base + kErrBytes + lat;
        g.ds_part = (int64_t *)p;
        g.ds_psum = (double *)(p + align_up((int64_t)DS_PARTS * (ds->n_bins + 2) * 8));
        g.ds_hist = ds->hist;
        g.ds_counts = ds->counts;
        g.ds_sums = ds->sums;
        g.ds_min = ds->min_size;
        g.ds_rmax = ds->r_max;
        g.ds_nbins = ds->n_bins;
    }
    g.phi = (const float *)field;
    g.tkey = tkey;
    g.labels = labels;
    g.n_clusters = n_clusters;
    g.sizes = sizes;
    (void)hipGetLastError();
    hipEvent_t *ev = profile_events();
    if (launch_single(g, stream, ev, pk) != hipSuccess) return HK_ERR_HIP;
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_label(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, int32_t *labels,
             int64_t *n_clusters, int64_t *sizes, hipStream_t stream) {
    return label_one(phi, PK_GT0, 0, nx, ny, nz, periodic_mask, labels, n_clusters, sizes, stream);
}

int hk_label_droplets(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, int32_t *labels,
                      int64_t *n_clusters, int64_t *sizes, int64_t min_size, double r_max, int32_t n_bins,
                      int64_t *hist, int64_t *counts, double *sums, hipStream_t stream) {
    if (!hist || !counts || !sums) return HK_ERR_INVALID_ARG;
    if (n_bins < 1 || n_bins > DS_MAXBINS || !(r_max > 0.0) || !std::isfinite(r_max)) return HK_ERR_INVALID_ARG;
    const DsArgs ds{min_size, r_max, n_bins, hist, counts, sums};
    return label_one(phi, PK_GT0, 0, nx, ny, nz, periodic_mask, labels, n_clusters, sizes, stream, &ds);
}

int hk_label_pred(const void *field, int32_t predicate, float param, int32_t nx, int32_t ny, int32_t nz,
                  uint32_t periodic_mask, int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream) {
    uint32_t pb;
    std::memcpy(&pb, &param, sizeof pb);
    const bool nan = (pb & 0x7fffffffu) > 0x7f800000u;
    int pk;
    switch (predicate) {
        case HK_PRED_GT:
            if (nan) return HK_ERR_INVALID_ARG;
            // field > +-0 is the cluster condition itself: share its kernel
            pk = order_key(pb) == 0 ? PK_GT0 : PK_GT;
            break;
        case HK_PRED_EQ:
            if (nan) return HK_ERR_INVALID_ARG;
            pk = PK_EQ;
            break;
        case HK_PRED_U8: pk = PK_U8; break;
        default: return HK_ERR_INVALID_ARG;
    }
    return label_one(field, pk, order_key(pb), nx, ny, nz, periodic_mask, labels, n_clusters, sizes, stream);
}

// ------------------------------------------------------------ incremental

struct hk_incr {
    int device = 0;
    hk::Geo g;           // geometry and workspace pointers (caller buffers unset)
    char *base = nullptr;
    bool primed = false; // a labelling has run: the saved tables are valid
};

int hk_incr_create(int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, hk_incr **out) {
    if (!out) return HK_ERR_INVALID_ARG;
    *out = nullptr;
    int rc = check_shape(nx, ny, nz, periodic_mask);
    if (rc != HK_OK) return rc;
    Geo g;
    rc = plan_lattice(nx, ny, nz, periodic_mask, &g);
    if (rc != HK_OK) return rc;
    const Layout L = layout_of(g, 0);
    const int64_t words = (int64_t)g.nb * g.R, nodes = (int64_t)g.nb * g.cap;
    const int64_t o_nsize0 = kErrBytes + L.total;
    const int64_t o_rootw0 = align_up(o_nsize0 + nodes * 4);
    const int64_t total = align_up(o_rootw0 + words * 8);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    void *p = nullptr;
    if (hipMalloc(&p, (size_t)total) != hipSuccess) return HK_ERR_HIP;
    if (hipMemset(p, 0, (size_t)kErrBytes) != hipSuccess) {
        (void)hipFree(p);
        return HK_ERR_HIP;
    }
    hk_incr *st = new hk_incr;
    st->device = dev;
    st->base = (char *)p;
    st->g = g;
    st->g.err = (int32_t *)st->base;
    bind(&st->g, st->base + kErrBytes, L);
    st->g.nsize0 = (int32_t *)(st->base + o_nsize0);
    st->g.rootw0 = (uint64_t *)(st->base + o_rootw0);
    *out = st;
    return HK_OK;
}

int hk_incr_label(hk_incr *st, const float *phi, int32_t *labels, int64_t *n_clusters, int64_t *sizes,
                  int64_t *relabelled, hipStream_t stream) {
    if (!st || !phi || !labels || !n_clusters) return HK_ERR_INVALID_ARG;
    if ((const void *)labels == (const void *)phi) return HK_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    if (dev != st->device) return HK_ERR_INVALID_ARG;
    Geo g = st->g;
    g.phi = phi;
    g.tkey = 0;
    g.labels = labels;
    g.n_clusters = n_clusters;
    g.sizes = sizes;
    g.incr = st->primed ? 2 : 1;
    g.nchanged = relabelled;
    (void)hipGetLastError();
    if (relabelled) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, stream, relabelled);
    hipEvent_t *ev = profile_events();
    if (launch_single(g, stream, ev, PK_GT0) != hipSuccess) return HK_ERR_HIP;
    st->primed = true;
    return HK_OK;
}

int hk_incr_device_error(hk_incr *st, hipStream_t stream, int32_t *code) {
    if (!st) return HK_ERR_INVALID_ARG;
    if (hipStreamSynchronize(stream) != hipSuccess) return HK_ERR_HIP;
    int32_t v = 0;
    if (hipMemcpy(&v, st->g.err, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return HK_ERR_HIP;
    if (code) *code = v;
    if (v && hipMemset(st->g.err, 0, sizeof v) != hipSuccess) return HK_ERR_HIP;
    return v ? HK_ERR_DEVICE : HK_OK;
}

void hk_incr_destroy(hk_incr *st) {
    if (!st) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(st->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(st->base);
    (void)hipSetDevice(cur);
    delete st;
}

int hk_reserve(int64_t bytes, hipStream_t stream) {
    if (bytes < 0) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace *ws = nullptr;
    const int rc = get_workspace(stream, bytes, &ws);
    if (rc != HK_OK) return rc;
    return ensure_capture_arena();
}

void hk_release(void) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        if (!kv.second.base) continue;
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        (void)hipFree(kv.second.base);
    }
    g_ws.clear();
    release_batched();
    (void)hipSetDevice(cur);
}

const char *hk_status_string(int status) {
    switch (status) {
        case HK_OK: return "HK_OK";
        case HK_ERR_INVALID_ARG: return "HK_ERR_INVALID_ARG: invalid argument";
        case HK_ERR_TOO_LARGE: return "HK_ERR_TOO_LARGE: lattice too large";
        case HK_ERR_NO_WORKSPACE: return "HK_ERR_NO_WORKSPACE: workspace must be reserved before capture";
        case HK_ERR_HIP: return "HK_ERR_HIP: HIP runtime or launch failure";
        case HK_ERR_DEVICE: return "HK_ERR_DEVICE: a device-side check fired";
        case HK_ERR_TIMEOUT: return "HK_ERR_TIMEOUT: time limit reached";
        default: return "unknown hk status";
    }
}

int hk_set_brick(int32_t by, int32_t bz) {
    if (by == 0 && bz == 0) {
        std::lock_guard<std::mutex> lk(g_brick_mu);
        g_force_by = g_force_bz = 0;
        return HK_OK;
    }
    if (!is_pow2(by) || !is_pow2(bz) || by * bz > RMAX) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_brick_mu);
    g_force_by = by;
    g_force_bz = bz;
    return HK_OK;
}

int hk_get_brick(int32_t nx, int32_t ny, int32_t nz, int32_t *by, int32_t *bz) {
    if (!by || !bz) return HK_ERR_INVALID_ARG;
    const int rc = check_shape(nx, ny, nz, 0);
    if (rc != HK_OK) return rc;
    Geo g;
    const int pr = plan_lattice(nx, ny, nz, 0, &g);
    if (pr != HK_OK) return pr;
    *by = g.BY;
    *bz = g.BZ;
    return HK_OK;
}

int hk_set_brick_for_shape(int32_t nx, int32_t ny, int32_t nz, int32_t by, int32_t bz) {
    const int rc = check_shape(nx, ny, nz, 0);
    if (rc != HK_OK) return rc;
    if (by == 0 && bz == 0) {
        std::lock_guard<std::mutex> lk(g_brick_mu);
        g_tuned.erase(bucket_of(nx, ny, nz));
        return HK_OK;
    }
    if (!is_pow2(by) || !is_pow2(bz) || by * bz > RMAX) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_brick_mu);
    g_tuned[bucket_of(nx, ny, nz)] = {by, bz};
    return HK_OK;
}

int hk_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    return HK_OK;
}

int hk_profile_read(float *ms, int32_t n, int32_t *calls) {
    if (!ms || n < 0) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < n; ++i) ms[i] = 0.0f;
    const int32_t c = (int32_t)g_prof_calls.size();
    int rc = HK_OK;
    for (auto &ev : g_prof_calls) {
        if (hipEventSynchronize(ev[kPhases]) != hipSuccess) rc = HK_ERR_HIP;
        for (int i = 0; i < kPhases && i < n && rc == HK_OK; ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) rc = HK_ERR_HIP;
            ms[i] += t;
        }
        for (auto e : ev) g_prof_pool.push_back(e);
    }
    g_prof_calls.clear();
    if (calls) *calls = c;
    return rc;
}

int32_t hk_phase_count(void) { return kPhases; }

const char *hk_phase_name(int32_t i) { return (i >= 0 && i < kPhases) ? kPhaseNames[i] : ""; }

int hk_debug_counters(hipStream_t stream, int64_t *counts, int32_t n) {
    if (!counts || n < 0) return HK_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    uint32_t v[DBG_N] = {0, 0, 0, 0};
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        auto it = g_ws.find({dev, stream});
        if (it != g_ws.end() && it->second.base) {
            if (hipStreamSynchronize(stream) != hipSuccess) return HK_ERR_HIP;
            uint32_t *d = dbg_counters(it->second.base);
            if (hipMemcpy(v, d, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return HK_ERR_HIP;
            if (hipMemset(d, 0, sizeof v) != hipSuccess) return HK_ERR_HIP;
        }
    }
    for (int i = 0; i < n; ++i) counts[i] = i < DBG_N ? (int64_t)v[i] : 0;
    return HK_OK;
}

int hk_device_error(hipStream_t stream, int32_t *code) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    int32_t v = 0;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        auto it = g_ws.find({dev, stream});
        if (it == g_ws.end() || !it->second.base) {
            if (code) *code = 0;
            return HK_OK;
        }
        if (hipStreamSynchronize(stream) != hipSuccess) return HK_ERR_HIP;
        if (hipMemcpy(&v, it->second.base, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return HK_ERR_HIP;
        if (v != 0 && hipMemset(it->second.base, 0, sizeof(v)) != hipSuccess) return HK_ERR_HIP;
    }
    if (code) *code = v;
    return v ? HK_ERR_DEVICE : HK_OK;
}

}  // extern "C"
