// Batched labelling: many lattices of any shapes in one stream-ordered
// group of launches.
//
// Each phase of the path is ONE kernel over the items (bricks, blocks of
// rows) of every job of the batch: workgroup w of phase p runs item
// w - itoff[p][j] of the job j whose item range holds w.  The phases of a job
// depend on each other only through the kernel boundaries, where the device
// makes every write of one phase visible to the next.  (A single persistent
// launch with per-item completion counters needs a device-scope release and
// acquire around every item; with one L2 per XCD those are L2 write-backs
// and invalidations, which cost more than the items themselves.)
//
// The job table (per-job geometry and workspace pointers, per-phase item
// offsets) is uploaded with one host-to-device copy from pinned memory right
// before the launches, so a hipGraph capture of one call holds one copy node
// and one kernel node per phase.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/hk.h"
#include "hk_device.h"
#include "hk_launch.h"

namespace hk {

// eight waves per SIMD, four bricks per CU, as for the single-lattice kernel
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8))) void kb_local(GroupView v) {
    __shared__ LdsBrick s;
    int i;
    const Geo &g = locate(v, 0, blockIdx.x, &i);
    phase_local(g, i, s);
}

__global__ __launch_bounds__(WG_MERGE) __attribute__((amdgpu_waves_per_eu(8))) void kb_merge(GroupView v) {
    __shared__ MergeLds m;
    int i;
    const Geo &g = locate(v, 1, blockIdx.x, &i);
    phase_merge(g, i, m);
}

__global__ __launch_bounds__(WG_NODES) void kb_roots(GroupView v) {
    __shared__ int32_t hash[2 * HT];
    __shared__ uint64_t rbits[RMAX];
    int i;
    const Geo &g = locate(v, 2, blockIdx.x, &i);
    phase_roots(g, i, 1, hash, rbits);
}

__global__ __launch_bounds__(WG) void kb_rowsum(GroupView v) {
    __shared__ int32_t tmp[32];
    int i;
    const Geo &g = locate(v, 3, blockIdx.x, &i);
    phase_rowsum(g, i, tmp);
}

__global__ __launch_bounds__(WG) void kb_scanblk(GroupView v) {
    __shared__ int32_t tmp[32];
    int i;
    const Geo &g = locate(v, 4, blockIdx.x, &i);
    phase_scanblk(g, tmp);
}

__global__ __launch_bounds__(WG) void kb_rowpre(GroupView v) {
    __shared__ int32_t tmp[32];
    int i;
    const Geo &g = locate(v, 5, blockIdx.x, &i);
    phase_rowpre(g, i, tmp);
}


__global__ __launch_bounds__(WG_RANK) __attribute__((amdgpu_waves_per_eu(8))) void kb_rank(GroupView v) {
    int i;
    const Geo &g = locate(v, 6, blockIdx.x, &i);
    phase_rank(g, i, 1);
}

__global__ __launch_bounds__(WG) void kb_write(GroupView v) {
    __shared__ LdsBrick s;
    int i;
    const Geo &g = locate(v, 7, blockIdx.x, &i);
    phase_write(g, i, s);
}

static_assert(NPH == kPhases, "one grouped kernel per phase of the single-lattice path");

// ------------------------------------------------------------------- host

int plan_lattice_ext(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g);
int64_t lattice_bytes(const Geo &g);
void bind_lattice(Geo *g, char *base);
int acquire_workspace(hipStream_t st, int64_t bytes, char **base, int32_t **err);
uint32_t *workspace_dbg(int32_t *err);
std::mutex &workspace_mutex();

namespace {

int64_t al(int64_t v) { return (v + 255) / 256 * 256; }

struct TableLayout {
    int64_t jobs, itoff, total;
};

TableLayout table_layout(int n) {
    TableLayout t;
    int64_t o = 0;
    t.jobs = o;
    o = al(o + (int64_t)n * sizeof(Geo));
    t.itoff = o;
    o = al(o + (int64_t)NPH * (n + 1) * 4);
    t.total = o;
    return t;
}

int items_of(const Geo &g, int p) {
    switch (p) {
        case 3:
        case 5: return g.nblk;
        case 4: return 1;
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
// that last read a block has completed
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

// upload the table image to `table` on `stream` from pinned memory
int upload_table(const std::vector<char> &img, char *table, hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return HK_ERR_HIP;
    const int64_t n = (int64_t)img.size();
    if (cs != hipStreamCaptureStatusNone) {
        if (!g_arena.base || g_arena.used + al(n) > g_arena.size) return HK_ERR_NO_WORKSPACE;
        char *host = g_arena.base + g_arena.used;
        g_arena.used += al(n);
        std::memcpy(host, img.data(), (size_t)n);
        return hipMemcpyAsync(table, host, (size_t)n, hipMemcpyHostToDevice, stream) == hipSuccess ? HK_OK
                                                                                                   : HK_ERR_HIP;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    Staging &sg = g_stage[{dev, stream}];
    const int k = sg.next;
    sg.next = (k + 1) % 4;
    if (sg.used[k] && hipEventSynchronize(sg.ev[k]) != hipSuccess) return HK_ERR_HIP;
    if (sg.cap[k] < n) {
        if (sg.host[k]) (void)hipHostFree(sg.host[k]);
        sg.host[k] = nullptr;
        sg.cap[k] = 0;
        if (hipHostMalloc(&sg.host[k], (size_t)n, hipHostMallocDefault) != hipSuccess) return HK_ERR_HIP;
        sg.cap[k] = n;
    }
    if (!sg.ev[k] && hipEventCreateWithFlags(&sg.ev[k], hipEventDisableTiming) != hipSuccess) return HK_ERR_HIP;
    std::memcpy(sg.host[k], img.data(), (size_t)n);
    if (hipMemcpyAsync(table, sg.host[k], (size_t)n, hipMemcpyHostToDevice, stream) != hipSuccess) return HK_ERR_HIP;
    if (hipEventRecord(sg.ev[k], stream) != hipSuccess) return HK_ERR_HIP;
    sg.used[k] = true;
    return HK_OK;
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

// Enqueue the table upload and the eight grouped kernels of a validated
// batch; `ws` holds at least the bytes validate_and_plan reported.  The
// caller holds the workspace mutex (it guards the staging ring).
// Job j's device-check word is at err + j * err_stride bytes (stride 0: one
// word for the whole batch).
int enqueue_batched(const hk_job *jobs, int n_jobs, const std::vector<Geo> &geos, char *ws, int32_t *err,
                    int64_t err_stride, uint32_t *dbg, hipStream_t stream) {
    const TableLayout tl = table_layout(n_jobs);
    std::vector<char> img((size_t)tl.total, 0);
    int32_t *itoff = (int32_t *)(img.data() + tl.itoff);
    int64_t items[NPH];
    for (int p = 0; p < NPH; ++p) {
        int32_t *off = itoff + p * (n_jobs + 1);
        int64_t acc = 0;
        for (int j = 0; j < n_jobs; ++j) {
            off[j] = (int32_t)acc;
            acc += items_of(geos[j], p);
            if (acc > INT32_MAX) return HK_ERR_TOO_LARGE;
        }
        off[n_jobs] = (int32_t)acc;
        items[p] = acc;
    }
    char *table = ws;
    char *cursor = ws + tl.total;
    Geo *hj = (Geo *)(img.data() + tl.jobs);
    for (int j = 0; j < n_jobs; ++j) {
        Geo g = geos[j];
        bind_lattice(&g, cursor);
        cursor += al(lattice_bytes(g));
        g.err = (int32_t *)((char *)err + (int64_t)j * err_stride);
        g.dbg = dbg;
        g.phi = jobs[j].phi;
        g.labels = jobs[j].labels;
        g.n_clusters = jobs[j].n_clusters;
        g.sizes = jobs[j].sizes;
        hj[j] = g;
    }
    const int rc = upload_table(img, table, stream);
    if (rc != HK_OK) return rc;

    GroupView v;
    v.jobs = (ConstGeo *)(table + tl.jobs);
    v.itoff = (ConstI32 *)(table + tl.itoff);
    v.njobs = n_jobs;
    const dim3 blk(WG), small(WG_NODES);
    (void)hipGetLastError();
    hipLaunchKernelGGL(kb_local, dim3((unsigned)items[0]), blk, 0, stream, v);
    hipLaunchKernelGGL(kb_merge, dim3((unsigned)items[1]), dim3(WG_MERGE), 0, stream, v);
    hipLaunchKernelGGL(kb_roots, dim3((unsigned)items[2]), small, 0, stream, v);
    hipLaunchKernelGGL(kb_rowsum, dim3((unsigned)items[3]), blk, 0, stream, v);
    hipLaunchKernelGGL(kb_scanblk, dim3((unsigned)items[4]), blk, 0, stream, v);
    hipLaunchKernelGGL(kb_rowpre, dim3((unsigned)items[5]), blk, 0, stream, v);
    hipLaunchKernelGGL(kb_rank, dim3((unsigned)items[6]), dim3(WG_RANK), 0, stream, v);
    hipLaunchKernelGGL(kb_write, dim3((unsigned)items[7]), blk, 0, stream, v);
    return hipGetLastError() == hipSuccess ? HK_OK : HK_ERR_HIP;
}

// validation and workspace size of a batch, exposed to the server
int plan_batched(const hk_job *jobs, int n_jobs, std::vector<Geo> *geos, int64_t *bytes) {
    return validate_and_plan(jobs, n_jobs, true, geos, bytes);
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
    std::lock_guard<std::mutex> lk(workspace_mutex());
    char *base = nullptr;
    int32_t *err = nullptr;
    rc = acquire_workspace(stream, bytes, &base, &err);
    if (rc != HK_OK) return rc;
    return enqueue_batched(jobs, n_jobs, geos, base, err, 0, workspace_dbg(err), stream);
}

}  // extern "C"
