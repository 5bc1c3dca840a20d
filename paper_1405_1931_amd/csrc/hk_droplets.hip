// Droplet-size statistics (Sec. 5) of a sizes array: the count, the summed
// size, the histogram of the radius of the sphere of the same volume and the
// sums of R, R^2, R^3 of the clusters of at least min_size sites.  The
// binning and the per-cluster terms are those of the rank phase's fused form
// (ds_init, ds_add): the same bins, exactly, for the same sizes.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "../../include/hk.h"
#include "hk_device.h"

namespace hk {
namespace {

constexpr int DS_WG = 256;

__global__ __launch_bounds__(DS_WG) void k_ds_zero(int64_t *hist, int n_bins, int64_t *counts, double *sums) {
    for (int i = blockIdx.x * DS_WG + threadIdx.x; i < n_bins; i += gridDim.x * DS_WG) hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) counts[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 3) sums[threadIdx.x] = 0.0;
}

__device__ __forceinline__ double block_sum_f64(double v, double *tmp) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) tmp[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < DS_WG / 64; ++i) t += tmp[i];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(DS_WG) void k_ds_stats(const int64_t *sizes, const int64_t *nk, int64_t cap,
                                                    int64_t min_size, double r_max, int n_bins, int64_t *hist,
                                                    int64_t *counts, double *sums) {
    __shared__ double T[DS_MAXBINS];
    __shared__ int32_t h[DS_MAXBINS];
    __shared__ double tmp[DS_WG / 64];
    __shared__ DsTab tab;
    ds_init(r_max, n_bins, T, h, &tab, threadIdx.x, DS_WG);
    __syncthreads();
    const int64_t k = min(*nk, cap);
    DsAcc a;
    for (int64_t i = (int64_t)blockIdx.x * DS_WG + threadIdx.x; i < k; i += (int64_t)gridDim.x * DS_WG)
        ds_add(a, T, h, &tab, n_bins, min_size, sizes[i]);
    // cnt and ssum fit a double exactly up to 2^53, far above any lattice here
    const double tc = block_sum_f64((double)a.cnt, tmp);
    const double ts = block_sum_f64((double)a.ssum, tmp);
    const double t1 = block_sum_f64(a.sr, tmp);
    const double t2 = block_sum_f64(a.sr2, tmp);
    const double t3 = block_sum_f64(a.sr3, tmp);
    for (int i = threadIdx.x; i < n_bins; i += DS_WG)
        if (h[i]) atomicAdd((unsigned long long *)(hist + i), (unsigned long long)h[i]);
    if (threadIdx.x == 0 && tc > 0.0) {
        atomicAdd((unsigned long long *)(counts + 0), (unsigned long long)tc);
        atomicAdd((unsigned long long *)(counts + 1), (unsigned long long)ts);
        atomicAdd(sums + 0, t1);
        atomicAdd(sums + 1, t2);
        atomicAdd(sums + 2, t3);
    }
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" int hk_droplet_stats(const int64_t *sizes, const int64_t *n_clusters, int64_t max_clusters,
                                int64_t min_size, double r_max, int32_t n_bins, int64_t *hist, int64_t *counts,
                                double *sums, hipStream_t stream) {
    if (!sizes || !n_clusters || !hist || !counts || !sums) return HK_ERR_INVALID_ARG;
    if (max_clusters < 0 || n_bins < 1 || n_bins > DS_MAXBINS || !(r_max > 0.0) || !isfinite(r_max))
        return HK_ERR_INVALID_ARG;
    const int groups = (int)std::min<int64_t>(std::max<int64_t>(1, (max_clusters + DS_WG - 1) / DS_WG), 1024);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_ds_zero, dim3((n_bins + DS_WG - 1) / DS_WG), dim3(DS_WG), 0, stream, hist, n_bins, counts,
                       sums);
    hipLaunchKernelGGL(k_ds_stats, dim3(groups), dim3(DS_WG), 0, stream, sizes, n_clusters, max_clusters, min_size,
                       r_max, n_bins, hist, counts, sums);
    return hipGetLastError() == hipSuccess ? HK_OK : HK_ERR_HIP;
}
