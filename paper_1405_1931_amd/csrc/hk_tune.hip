// Brick-shape autotuner.
//
// The brick (64 x BY x BZ sites, one workgroup) is the unit of the local
// labelling, of the face merge and of the relabel; its shape trades node
// count (face area) against bricks in flight.  The tuner times every
// candidate shape on the caller's own lattice (or batch) with HIP events on
// the caller's stream, keeps the fastest, and installs it for the size bucket
// (power-of-two edges) of the lattice, or of every lattice of the batch, in
// the table that brick choice consults before its size heuristic.  The
// table can be written to and read from a text file.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/hk.h"
#include "hk_device.h"

namespace hk {

void brick_forced(int *by, int *bz);
void brick_force(int by, int bz);
std::vector<std::pair<uint32_t, std::pair<int, int>>> brick_table();
void brick_table_set(uint32_t bucket, int by, int bz);
uint32_t brick_bucket(int nx, int ny, int nz);

namespace {

int ceil_pow2(int v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

// power-of-two shapes that fit the lattice, with as many rows as it allows
// up to RMAX and at least min(64, what the lattice allows)
std::vector<std::pair<int, int>> candidates(int ny, int nz) {
    const int my = std::min(ceil_pow2(ny), RMAX), mz = std::min(ceil_pow2(nz), RMAX);
    const int rmin = std::min(64, my * mz);
    std::vector<std::pair<int, int>> c;
    for (int y = 1; y <= my; y <<= 1)
        for (int z = 1; z <= mz; z <<= 1)
            if (y * z <= RMAX && y * z >= rmin) c.push_back({y, z});
    return c;
}

std::mutex g_tune_mu;  // one tuning run at a time (it overrides the forced brick)

// mean ms of `reps` runs of fn() on `st`, after one untimed run
template <class F>
int time_runs(hipStream_t st, int reps, F fn, float *ms) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return HK_ERR_HIP;
    int rc = fn();
    if (rc == HK_OK && hipEventRecord(a, st) != hipSuccess) rc = HK_ERR_HIP;
    for (int i = 0; rc == HK_OK && i < reps; ++i) rc = fn();
    if (rc == HK_OK && hipEventRecord(b, st) != hipSuccess) rc = HK_ERR_HIP;
    if (rc == HK_OK && hipEventSynchronize(b) != hipSuccess) rc = HK_ERR_HIP;
    float t = 0.0f;
    if (rc == HK_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = HK_ERR_HIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / (float)reps;
    return rc;
}

// time each candidate with fn(); install the best for every bucket given
template <class F>
int tune(const std::vector<std::pair<int, int>> &cand, const std::vector<uint32_t> &buckets, int reps,
         hipStream_t st, F fn, int32_t *by, int32_t *bz, float *ms) {
    if (reps < 1 || cand.empty()) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int fy = 0, fz = 0;
    brick_forced(&fy, &fz);
    int best = -1;
    float best_ms = 0.0f;
    int rc = HK_OK;
    for (size_t i = 0; i < cand.size(); ++i) {
        brick_force(cand[i].first, cand[i].second);
        float t = 0.0f;
        rc = time_runs(st, reps, fn, &t);
        if (rc != HK_OK) break;
        if (best < 0 || t < best_ms) {
            best = (int)i;
            best_ms = t;
        }
    }
    brick_force(fy, fz);
    if (rc != HK_OK) return rc;
    for (uint32_t b : buckets) brick_table_set(b, cand[best].first, cand[best].second);
    if (by) *by = cand[best].first;
    if (bz) *bz = cand[best].second;
    if (ms) *ms = best_ms;
    // leave the outputs holding a result of the chosen shape
    return fn();
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" {

int hk_autotune(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, int32_t *labels,
                int64_t *n_clusters, int64_t *sizes, int32_t reps, hipStream_t stream, int32_t *by, int32_t *bz,
                float *ms) {
    if (nx < 1 || ny < 1 || nz < 1 || periodic_mask > 7u) return HK_ERR_INVALID_ARG;
    if ((int64_t)nx * ny * nz > INT32_MAX) return HK_ERR_TOO_LARGE;
    if (!phi || !labels || !n_clusters) return HK_ERR_INVALID_ARG;
    auto fn = [&] { return hk_label(phi, nx, ny, nz, periodic_mask, labels, n_clusters, sizes, stream); };
    return tune(candidates(ny, nz), {brick_bucket(nx, ny, nz)}, reps, stream, fn, by, bz, ms);
}

int hk_autotune_batched(const hk_job *jobs, int32_t n_jobs, int32_t reps, hipStream_t stream, int32_t *by,
                        int32_t *bz, float *ms) {
    if (n_jobs < 1 || !jobs) return HK_ERR_INVALID_ARG;
    int my = 1, mz = 1;
    std::vector<uint32_t> buckets;
    for (int j = 0; j < n_jobs; ++j) {
        const hk_job &b = jobs[j];
        if (b.nx < 1 || b.ny < 1 || b.nz < 1 || b.periodic_mask > 7u) return HK_ERR_INVALID_ARG;
        if ((int64_t)b.nx * b.ny * b.nz > INT32_MAX) return HK_ERR_TOO_LARGE;
        my = std::max(my, b.ny);
        mz = std::max(mz, b.nz);
        buckets.push_back(brick_bucket(b.nx, b.ny, b.nz));
    }
    auto fn = [&] { return hk_label_batched(jobs, n_jobs, stream); };
    return tune(candidates(my, mz), buckets, reps, stream, fn, by, bz, ms);
}

int hk_tune_save(const char *path) {
    if (!path) return HK_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return HK_ERR_INVALID_ARG;
    std::fprintf(f, "# log2(nx) log2(ny) log2(nz) by bz\n");
    for (const auto &e : brick_table())
        std::fprintf(f, "%u %u %u %d %d\n", e.first & 0xFFu, (e.first >> 8) & 0xFFu, (e.first >> 16) & 0xFFu,
                     e.second.first, e.second.second);
    const bool ok = std::fclose(f) == 0;
    return ok ? HK_OK : HK_ERR_INVALID_ARG;
}

int hk_tune_load(const char *path) {
    if (!path) return HK_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return HK_ERR_INVALID_ARG;
    std::vector<std::pair<uint32_t, std::pair<int, int>>> rows;
    char line[256];
    int rc = HK_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        unsigned lx, ly, lz;
        int y, z;
        if (std::sscanf(line, "%u %u %u %d %d", &lx, &ly, &lz, &y, &z) != 5 || lx > 31 || ly > 31 || lz > 31 ||
            y < 1 || z < 1 || (y & (y - 1)) || (z & (z - 1)) || y * z > RMAX) {
            rc = HK_ERR_INVALID_ARG;
            break;
        }
        rows.push_back({lx | (ly << 8) | (lz << 16), {y, z}});
    }
    std::fclose(f);
    if (rc != HK_OK) return rc;  // nothing installed from a malformed file
    for (const auto &r : rows) brick_table_set(r.first, r.second.first, r.second.second);
    return HK_OK;
}

}  // extern "C"
