// Kernels of the single-lattice path: one workgroup per brick (or per block
// of WG lattice rows) and one launch per phase, all on the caller's stream.
#include <algorithm>

#include "hk_device.h"
#include "hk_launch.h"

namespace hk {

// Four bricks per CU need eight waves per SIMD: the LDS allows four (40 KB
// each), and the compiler is held to the scalar registers of one of eight
// waves (78; the values that no longer fit move to vector register lanes).
// Left free it uses more and three bricks run per CU, which measured 15-35 %
// slower at 1024^3.
template <int PK>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8))) void k_local(Geo g) {
    __shared__ LdsBrick s;
    phase_local<PK>(g, blockIdx.x, s);
}

__global__ __launch_bounds__(WG_MERGE) __attribute__((amdgpu_waves_per_eu(8))) void k_merge(Geo g) {
    __shared__ MergeLds m;
    phase_merge(g, blockIdx.x, m);
}

constexpr int ROOTS_BRICKS = ROOTS_MAX;  // bricks per workgroup of the roots phase

__global__ __launch_bounds__(WG_NODES) void k_roots(Geo g) {
    __shared__ int32_t hash[2 * HT];
    __shared__ uint64_t rbits[ROOTS_MAX * RMAX];
    phase_roots(g, blockIdx.x * ROOTS_BRICKS, ROOTS_BRICKS, hash, rbits);
}

__global__ __launch_bounds__(WG) void k_rowsum(Geo g) {
    __shared__ int32_t tmp[32];
    phase_rowsum(g, blockIdx.x, tmp);
    if (g.ds_part) ds_clear(g, blockIdx.x, gridDim.x);  // hk_label_droplets: before the rank phase
}

__global__ __launch_bounds__(WG) void k_scanblk(Geo g) {
    __shared__ int32_t tmp[32];
    phase_scanblk(g, tmp);
}

__global__ __launch_bounds__(WG) void k_rowpre(Geo g) {
    __shared__ int32_t tmp[32];
    phase_rowpre(g, blockIdx.x, tmp);
}


// node labels carry little work per brick and no LDS: small workgroups keep
// eight bricks per CU in flight
__global__ __launch_bounds__(WG_RANK) __attribute__((amdgpu_waves_per_eu(8))) void k_rank(Geo g) {
    const int b = xcd_brick_rank(g, blockIdx.x);
    if (b >= 0) phase_rank(g, b, min(RANK_BRICKS, g.nbx - b % g.nbx));
}

// the same, gathering the droplet statistics (hk_label_droplets)
__global__ __launch_bounds__(WG_RANK) __attribute__((amdgpu_waves_per_eu(8))) void k_rank_ds(Geo g) {
    __shared__ DsLds dl;
    const int b = xcd_brick_rank(g, blockIdx.x);
    if (b >= 0) phase_rank<true>(g, b, min(RANK_BRICKS, g.nbx - b % g.nbx), &dl);
}

// the outputs from the partial accumulators, one workgroup per column (a
// bin, the count, the summed size, then the three sums of R^k), its
// DS_PARTS threads one part each
static_assert(DS_PARTS == 256, "one thread per part");
__global__ __launch_bounds__(DS_PARTS) void k_ds_combine(Geo g) {
    __shared__ int64_t ri[DS_PARTS / 64];
    __shared__ double rd[DS_PARTS / 64];
    const int c = blockIdx.x, t = threadIdx.x, nc = g.ds_nbins + 2;
    if (c < nc) {
        int64_t v = g.ds_part[(int64_t)c * DS_PARTS + t];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((t & 63) == 0) ri[t >> 6] = v;
        __syncthreads();
        if (t == 0) {
            const int64_t s = ri[0] + ri[1] + ri[2] + ri[3];
            if (c < g.ds_nbins)
                g.ds_hist[c] = s;
            else
                g.ds_counts[c - g.ds_nbins] = s;
        }
    } else {
        double v = g.ds_psum[(c - nc) * DS_PARTS + t];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((t & 63) == 0) rd[t >> 6] = v;
        __syncthreads();
        if (t == 0) g.ds_sums[c - nc] = (rd[0] + rd[1]) + (rd[2] + rd[3]);
    }
}

__global__ __launch_bounds__(WG) void k_write(Geo g) {
    __shared__ LdsBrick s;
    const int b = xcd_brick(g, blockIdx.x);
    if (b >= 0) phase_write(g, b, s);
}

__global__ void k_zero_i64(int64_t *p) {
    if (threadIdx.x == 0) *p = 0;
}

const char *const kPhaseNames[kPhases] = {"k_local", "k_merge", "k_roots", "k_rowsum",
                                          "k_scanblk", "k_rowpre", "k_rank", "k_write"};

hipError_t launch_single(const Geo &g, hipStream_t st, hipEvent_t *ev, int pk) {
    const dim3 blk(WG), small(WG_NODES);
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    switch (pk) {
        case PK_GT: hipLaunchKernelGGL(k_local<PK_GT>, dim3(g.nb), blk, 0, st, g); break;
        case PK_EQ: hipLaunchKernelGGL(k_local<PK_EQ>, dim3(g.nb), blk, 0, st, g); break;
        case PK_U8: hipLaunchKernelGGL(k_local<PK_U8>, dim3(g.nb), blk, 0, st, g); break;
        default: hipLaunchKernelGGL(k_local<PK_GT0>, dim3(g.nb), blk, 0, st, g); break;
    }
    mark(1);
    hipLaunchKernelGGL(k_merge, dim3(g.nb), dim3(WG_MERGE), 0, st, g);
    mark(2);
    hipLaunchKernelGGL(k_roots, dim3((unsigned)(((int64_t)g.nb + ROOTS_BRICKS - 1) / ROOTS_BRICKS)), small, 0, st, g);
    mark(3);
    hipLaunchKernelGGL(k_rowsum, dim3(g.nblk), blk, 0, st, g);
    mark(4);
    hipLaunchKernelGGL(k_scanblk, dim3(1), blk, 0, st, g);
    mark(5);
    hipLaunchKernelGGL(k_rowpre, dim3(g.nblk), blk, 0, st, g);
    mark(6);
    if (g.ds_part) {
        hipLaunchKernelGGL(k_rank_ds, dim3((unsigned)xcd_grid_rank(g)), dim3(WG_RANK), 0, st, g);
        hipLaunchKernelGGL(k_ds_combine, dim3((unsigned)(g.ds_nbins + 5)), dim3(DS_PARTS), 0, st, g);
    } else {
        hipLaunchKernelGGL(k_rank, dim3((unsigned)xcd_grid_rank(g)), dim3(WG_RANK), 0, st, g);
    }
    mark(7);
    hipLaunchKernelGGL(k_write, dim3((unsigned)xcd_grid(g)), blk, 0, st, g);
    mark(8);
    return hipGetLastError();
}

}  // namespace hk
