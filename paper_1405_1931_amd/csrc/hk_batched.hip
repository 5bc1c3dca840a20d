// Batched labelling: many lattices of any shapes in ONE persistent launch.
//
// Work items are (phase, job, item) triples laid out phase-major: all pack
// items of every job, then all local items, ... then all write items.
// Resident workgroups pop item indices from a global counter.  Before an
// item of phase p runs, the workgroup waits until every item of phase p-1 of
// the same job has finished (per-job, per-phase completion counters).  An
// item only ever waits for items with smaller indices, which were popped
// earlier by workgroups that are already running, so the queue always drains
// (the oldest unfinished item never waits).  Every wait is also bounded by a
// wall-clock limit that sets the sticky device error instead of hanging.
//
// The job table (per-job geometry and workspace pointers, item offsets,
// zeroed counters) is uploaded with one host-to-device copy from pinned
// memory right before the launch, so a hipGraph capture of one call holds
// exactly one copy node and one kernel node, and every replay starts from
// zeroed counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/hk.h"
#include "hk_device.h"

namespace hk {

__global__ __launch_bounds__(WG) void k_batched(BatchView v) {
    __shared__ LdsBrick s;
    __shared__ int s_item;
    persistent_loop(v, s, s_item);
}

// ------------------------------------------------------------------- host

int plan_lattice_ext(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g);
int64_t lattice_bytes(const Geo &g);
void bind_lattice(Geo *g, char *base);
int acquire_workspace(hipStream_t st, int64_t bytes, char **base, int32_t **err);
std::mutex &workspace_mutex();

namespace {

int64_t al(int64_t v) { return (v + 255) / 256 * 256; }

// bound on one dependency wait inside the persistent kernel: HK_WAIT_MS
// milliseconds (default 10 s), in ticks of the 100 MHz constant clock
uint64_t wait_ticks() {
    static uint64_t ticks = [] {
        uint64_t ms = 10000;
        if (const char *e = std::getenv("HK_WAIT_MS")) {
            const long v = std::atol(e);
            if (v > 0) ms = (uint64_t)v;
        }
        return ms * 100000ull;
    }();
    return ticks;
}

struct TableLayout {
    int64_t jobs, itoff, pstart, done, next, total;
};

TableLayout table_layout(int n) {
    TableLayout t;
    int64_t o = 0;
    t.jobs = o;
    o = al(o + (int64_t)n * sizeof(Geo));
    t.itoff = o;
    o = al(o + (int64_t)NPH * (n + 1) * 4);
    t.pstart = o;
    o = al(o + (NPH + 1) * 4);
    t.done = o;
    o = al(o + (int64_t)n * NPH * 4);
    t.next = o;
    o = al(o + 4);
    t.total = o;
    return t;
}

int items_of(const Geo &g, int p) {
    switch (p) {
        case 4:
        case 6: return g.nblk;
        case 5: return 1;
        default: return g.nb;
    }
}

int validate_and_plan(const hk_job *jobs, int n, bool need_ptrs, std::vector<Geo> *geos, int64_t *bytes) {
    geos->resize(n);
    int64_t total = 0;
    for (int j = 0; j < n; ++j) {
        const hk_job &b = jobs[j];
        if (need_ptrs) {
            if (!b.phi || !b.labels || !b.n_clusters) return HK_ERR_INVALID_ARG;
            if ((const void *)b.phi == (const void *)b.labels) return HK_ERR_INVALID_ARG;
        }
        if (b.nx < 1 || b.ny < 1 || b.nz < 1 || b.periodic_mask > 7u) return HK_ERR_INVALID_ARG;
        if ((int64_t)b.nx * b.ny * b.nz > INT32_MAX) return HK_ERR_TOO_LARGE;
        const int rc = plan_lattice_ext(b.nx, b.ny, b.nz, b.periodic_mask, &(*geos)[j]);
        if (rc != HK_OK) return rc;
        total = al(total + lattice_bytes((*geos)[j]));
    }
    *bytes = total + table_layout(n).total;
    return HK_OK;
}

// pinned staging blocks for the job table: a small ring reused once the copy
// that last read a block has completed; blocks used under capture are kept
// for the lifetime of the library (a graph replays from them)
struct Staging {
    void *host[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t cap[4] = {0, 0, 0, 0};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool used[4] = {false, false, false, false};
    int next = 0;
};
std::map<std::pair<int, hipStream_t>, Staging> g_stage;

// pinned arena for the job tables of captured calls: allocated by
// hk_reserve (allocation is not allowed while a stream is captured), carved
// by captured calls, kept until hk_release because graphs replay from it
struct CaptureArena {
    char *base = nullptr;
    int64_t size = 0, used = 0;
};
CaptureArena g_arena;
constexpr int64_t kArenaBytes = 8ll << 20;

int grid_size() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched, WG, 0) != hipSuccess) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    const int v = std::max(1, per_cu) * std::max(1, cus);
    if (dev >= 0 && dev < 64) cached[dev] = v;
    return v;
}

}  // namespace

// called by hk_reserve (with the workspace mutex held)
int ensure_capture_arena() {
    if (g_arena.base) return HK_OK;
    void *p = nullptr;
    if (hipHostMalloc(&p, (size_t)kArenaBytes, hipHostMallocDefault) != hipSuccess) return HK_ERR_HIP;
    g_arena.base = (char *)p;
    g_arena.size = kArenaBytes;
    g_arena.used = 0;
    return HK_OK;
}

// called by hk_release (with the workspace mutex held, devices synchronised)
void release_batched() {
    for (auto &kv : g_stage) {
        for (int k = 0; k < 4; ++k) {
            if (kv.second.host[k]) (void)hipHostFree(kv.second.host[k]);
            if (kv.second.ev[k]) (void)hipEventDestroy(kv.second.ev[k]);
        }
    }
    g_stage.clear();
    if (g_arena.base) (void)hipHostFree(g_arena.base);
    g_arena = CaptureArena();
}

}  // namespace hk

using namespace hk;

extern "C" {

int64_t hk_batched_workspace_bytes(const hk_job *jobs, int32_t n_jobs) {
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return HK_ERR_INVALID_ARG;
    std::vector<Geo> geos;
    int64_t bytes = 0;
    const int rc = validate_and_plan(jobs, n_jobs, false, &geos, &bytes);
    if (rc != HK_OK) return rc;
    return bytes + 256;
}

int hk_label_batched(const hk_job *jobs, int32_t n_jobs, hipStream_t stream) {
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return HK_ERR_INVALID_ARG;
    if (n_jobs == 0) return HK_OK;
    std::vector<Geo> geos;
    int64_t bytes = 0;
    int rc = validate_and_plan(jobs, n_jobs, true, &geos, &bytes);
    if (rc != HK_OK) return rc;

    const TableLayout tl = table_layout(n_jobs);
    std::lock_guard<std::mutex> lk(workspace_mutex());
    char *base = nullptr;
    int32_t *err = nullptr;
    rc = acquire_workspace(stream, bytes, &base, &err);
    if (rc != HK_OK) return rc;
    char *table = base;
    char *cursor = base + tl.total;

    // host image of the table
    std::vector<char> img((size_t)tl.total, 0);
    Geo *hj = (Geo *)(img.data() + tl.jobs);
    int32_t *itoff = (int32_t *)(img.data() + tl.itoff);
    int32_t *pstart = (int32_t *)(img.data() + tl.pstart);
    int64_t items = 0;
    for (int p = 0; p < NPH; ++p) {
        pstart[p] = (int32_t)items;
        int32_t *off = itoff + p * (n_jobs + 1);
        int32_t acc = 0;
        for (int j = 0; j < n_jobs; ++j) {
            off[j] = acc;
            acc += items_of(geos[j], p);
        }
        off[n_jobs] = acc;
        items += acc;
        if (items > INT32_MAX / 2) return HK_ERR_TOO_LARGE;
    }
    pstart[NPH] = (int32_t)items;
    for (int j = 0; j < n_jobs; ++j) {
        Geo g = geos[j];
        bind_lattice(&g, cursor);
        cursor += al(lattice_bytes(g));
        g.err = err;
        g.phi = jobs[j].phi;
        g.labels = jobs[j].labels;
        g.n_clusters = jobs[j].n_clusters;
        g.sizes = jobs[j].sizes;
        hj[j] = g;
    }

    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return HK_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) {
        if (!g_arena.base || g_arena.used + tl.total > g_arena.size) return HK_ERR_NO_WORKSPACE;
        char *host = g_arena.base + g_arena.used;
        g_arena.used += tl.total;
        std::memcpy(host, img.data(), img.size());
        if (hipMemcpyAsync(table, host, (size_t)tl.total, hipMemcpyHostToDevice, stream) != hipSuccess)
            return HK_ERR_HIP;
    } else {
        int dev = 0;
        (void)hipGetDevice(&dev);
        Staging &sg = g_stage[{dev, stream}];
        const int k = sg.next;
        sg.next = (k + 1) % 4;
        if (sg.used[k] && hipEventSynchronize(sg.ev[k]) != hipSuccess) return HK_ERR_HIP;
        if (sg.cap[k] < tl.total) {
            if (sg.host[k]) (void)hipHostFree(sg.host[k]);
            sg.host[k] = nullptr;
            sg.cap[k] = 0;
            if (hipHostMalloc(&sg.host[k], (size_t)tl.total, hipHostMallocDefault) != hipSuccess) return HK_ERR_HIP;
            sg.cap[k] = tl.total;
        }
        if (!sg.ev[k] && hipEventCreateWithFlags(&sg.ev[k], hipEventDisableTiming) != hipSuccess) return HK_ERR_HIP;
        std::memcpy(sg.host[k], img.data(), img.size());
        if (hipMemcpyAsync(table, sg.host[k], (size_t)tl.total, hipMemcpyHostToDevice, stream) != hipSuccess)
            return HK_ERR_HIP;
        if (hipEventRecord(sg.ev[k], stream) != hipSuccess) return HK_ERR_HIP;
        sg.used[k] = true;
    }

    BatchView v;
    v.jobs = (ConstGeo *)(table + tl.jobs);
    v.itoff = (const int32_t *)(table + tl.itoff);
    v.pstart = (const int32_t *)(table + tl.pstart);
    v.done = (int32_t *)(table + tl.done);
    v.next = (int32_t *)(table + tl.next);
    v.err = err;
    v.njobs = n_jobs;
    v.total = (int32_t)items;
    v.wait_ticks = wait_ticks();
    const int grid = std::max(1, std::min<int>(grid_size(), (int)items));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_batched, dim3(grid), dim3(WG), 0, stream, v);
    if (hipGetLastError() != hipSuccess) return HK_ERR_HIP;
    return HK_OK;
}

}  // extern "C"
