// hk_label_noalloc: hk_label with its workspace in a fixed device array of
// the library, for callers that cannot allocate device memory (code under
// stream capture, tight serving loops).  Nothing is allocated: the
// workspace of a lattice is carved from `scratch`, a file-scope device
// array of kScratchBytes that every device the library runs on holds for
// the life of the process.  Host code never uses the array's name as an
// address (on the host it only names the symbol): the device address is
// looked up once per device with hipGetSymbolAddress and kept.
//
// Every call on one device shares that device's array and leaves its
// contents behind; the only word that must start at zero (the device-check
// word) is cleared by a one-thread kernel at the start of each call.  Calls
// that overlap on one device (different streams, or different host
// threads) race on the array: a caller serialises them.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/hk.h"
#include "hk_launch.h"

namespace hk {

int plan_lattice_one(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g);
int64_t lattice_bytes(const Geo &g);
void bind_lattice(Geo *g, char *base);

namespace {

constexpr int64_t kScratchBytes = 64ll << 20;
constexpr int64_t kCheckBytes = 256;  // the device-check word's block, then the lattice workspace

static __device__ __align__(256) char scratch[kScratchBytes];

__global__ void k_noalloc_begin(int32_t *check) {
    if (threadIdx.x == 0) *check = 0;
}

// a device-side check that fired during the call: K reads as minus its code
__global__ void k_noalloc_end(const int32_t *check, int64_t *n_clusters) {
    if (threadIdx.x == 0 && *check != 0) *n_clusters = -(int64_t)*check;
}

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch;  // device -> device address of `scratch`

// the device address of this device's `scratch`, looked up on first use
int scratch_base(char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HK_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return HK_ERR_HIP;
        }
        it = g_scratch.emplace(dev, (char *)p).first;
    }
    *out = it->second;
    return HK_OK;
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" int hk_label_noalloc(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
                                int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream) {
    if (!phi || !labels || !n_clusters) return HK_ERR_INVALID_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || periodic_mask > 7u) return HK_ERR_INVALID_ARG;
    if ((int64_t)nx * ny * nz > INT32_MAX) return HK_ERR_TOO_LARGE;
    if ((const void *)labels == (const void *)phi) return HK_ERR_INVALID_ARG;
    Geo g;
    int rc = plan_lattice_one(nx, ny, nz, periodic_mask, &g);
    if (rc != HK_OK) return rc;
    if (kCheckBytes + lattice_bytes(g) > kScratchBytes) return HK_ERR_TOO_LARGE;  // beyond the fixed scratch
    char *base = nullptr;
    rc = scratch_base(&base);
    if (rc != HK_OK) return rc;
    g.err = (int32_t *)base;
    g.dbg = nullptr;
    bind_lattice(&g, base + kCheckBytes);
    g.phi = phi;
    g.tkey = 0;
    g.labels = labels;
    g.n_clusters = n_clusters;
    g.sizes = sizes;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(64), 0, stream, g.err);
    if (launch_single(g, stream, nullptr, PK_GT0) != hipSuccess) return HK_ERR_HIP;
    hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(64), 0, stream, g.err, n_clusters);
    return hipGetLastError() == hipSuccess ? HK_OK : HK_ERR_HIP;
}
