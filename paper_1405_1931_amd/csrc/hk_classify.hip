// Interior/exterior decision for the clusters of a labelling (the last step
// of the Sec. 6 interior detection): every cluster site looks at its face
// neighbours; each neighbour outside every cluster (label 0) is a border
// pair, counted on the negative side if its proximity value I is < 0 and on
// the positive side if I > 0 (0 and NaN count for neither).  A cluster is
// inside when its negative pairs outnumber its positive ones, outside in the
// opposite case, undecided on a tie.
//
// The counts of a workgroup are summed per cluster in an LDS hash and added
// to the global counters once per (workgroup, cluster), so the exterior
// cluster, which borders every capsule, receives one global add per
// workgroup instead of one per border site.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/hk.h"

namespace hk {
namespace {

constexpr int CL_WG = 256;        // threads per workgroup
constexpr int CL_ROWS = 8;        // lattice rows per wave
constexpr int CL_HT = 1024;       // LDS hash slots per workgroup

// the side of a proximity value, decided on its bits so that no
// flush-to-zero mode changes it: -1 negative, +1 positive, 0 for +-0 / NaN
__device__ __forceinline__ int side_of(float v) {
    const uint32_t b = __float_as_uint(v);
    const uint32_t mag = b & 0x7fffffffu;
    if (mag == 0u || mag > 0x7f800000u) return 0;
    return (b >> 31) ? -1 : 1;
}

struct Dims {
    int32_t nx, ny, nz;
    uint32_t mask;
};

__global__ __launch_bounds__(CL_WG) void k_cls_zero(const int64_t *nk, int64_t cap, int64_t *neg, int64_t *pos) {
    const int64_t k = min(*nk, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
        neg[i] = 0;
        pos[i] = 0;
    }
}

// neighbour coordinate of c one step d along an axis of length n, or -1
// when there is none: off the lattice on a closed axis, the site itself on
// a periodic axis of length 1, and on a periodic axis of length 2 only the
// +1 step counts (both steps reach the same site: one pair)
__device__ __forceinline__ int step(int c, int d, int n, bool per) {
    if (n == 1 || (per && n == 2 && d < 0)) return -1;
    c += d;
    if (c < 0 || c >= n) {
        if (!per) return -1;
        c = c < 0 ? c + n : c - n;
    }
    return c;
}

// One wave takes one 64-site chunk of an x row at a time (lane = x), so the
// site and each of its six neighbour rows are coalesced row reads and no
// site index is ever divided; I is read only where a cluster site meets a
// membrane site.
__global__ __launch_bounds__(CL_WG) void k_cls_count(const float *I, const int32_t *labels, Dims D, const int64_t *nk,
                                                     int64_t cap, int64_t *neg, int64_t *pos) {
    __shared__ int32_t hkey[CL_HT];
    __shared__ int32_t hneg[CL_HT];
    __shared__ int32_t hpos[CL_HT];
    for (int i = threadIdx.x; i < CL_HT; i += CL_WG) {
        hkey[i] = 0;
        hneg[i] = 0;
        hpos[i] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwv = CL_WG / 64;
    const int k = (int)min(*nk, cap);
    const bool px = D.mask & 1u, py = D.mask & 2u, pz = D.mask & 4u;
    // a workgroup takes CL_ROWS * 4 consecutive rows r = (z, y) (so the y and
    // z neighbour rows it reads are read close together in time, from the
    // same XCD cache); wave w takes rows w, w + 4, ...; y and z advance with
    // a carry, so no row index is divided inside the loop
    const int rows = D.ny * D.nz;
    const int64_t first = (int64_t)blockIdx.x * CL_ROWS * nwv;
    const int rend = (int)min((int64_t)rows, first + CL_ROWS * nwv);
    int r = (int)(first + wv);
    int z = r / D.ny, y = r - z * D.ny;
    const int dz = nwv / D.ny, dy = nwv - dz * D.ny;
    const uint32_t plane = (uint32_t)D.ny * (uint32_t)D.nx;
    for (; r < rend; r += nwv) {
        const uint32_t rb = (uint32_t)r * (uint32_t)D.nx;  // < 2^31 sites
        const int ym = step(y, -1, D.ny, py), yp = step(y, 1, D.ny, py);
        const int zm = step(z, -1, D.nz, pz), zp = step(z, 1, D.nz, pz);
        // neighbour row bases (or none), wave-uniform
        const int64_t bym = ym < 0 ? -1 : (int64_t)rb + (int64_t)(ym - y) * D.nx;
        const int64_t byp = yp < 0 ? -1 : (int64_t)rb + (int64_t)(yp - y) * D.nx;
        const int64_t bzm = zm < 0 ? -1 : (int64_t)rb + (int64_t)(zm - z) * plane;
        const int64_t bzp = zp < 0 ? -1 : (int64_t)rb + (int64_t)(zp - z) * plane;
        for (int x0 = 0; x0 < D.nx; x0 += 64) {
            const int x = x0 + lane;
            int lab = 0, cn = 0, cp = 0;
            if (x < D.nx) {
                lab = labels[rb + x];
                if (lab > 0 && lab <= k) {
                    const int xm = step(x, -1, D.nx, px), xp = step(x, 1, D.nx, px);
                    const bool has[6] = {xm >= 0, xp >= 0, bym >= 0, byp >= 0, bzm >= 0, bzp >= 0};
                    const uint32_t nb[6] = {rb + xm, rb + xp, (uint32_t)bym + x, (uint32_t)byp + x,
                                            (uint32_t)bzm + x, (uint32_t)bzp + x};
                    int nl[6];
#pragma unroll
                    for (int d = 0; d < 6; ++d) nl[d] = has[d] ? labels[nb[d]] : 1;
#pragma unroll
                    for (int d = 0; d < 6; ++d) {
                        if (nl[d] != 0) continue;
                        const int sd = side_of(I[nb[d]]);
                        cn += sd < 0;
                        cp += sd > 0;
                    }
                }
            }
            // lanes of one cluster first sum their counts across the wave;
            // one lane per cluster then updates the workgroup's hash
            bool pending = (cn | cp) != 0;
            for (;;) {
                const uint64_t m = __ballot(pending);
                if (m == 0) break;
                const int leader = __builtin_ctzll(m);
                const int L = __shfl(lab, leader, 64);
                const bool mine = pending && lab == L;
                int sn = mine ? cn : 0, sp = mine ? cp : 0;
                for (int o = 32; o > 0; o >>= 1) {
                    sn += __shfl_xor(sn, o, 64);
                    sp += __shfl_xor(sp, o, 64);
                }
                if (mine) pending = false;
                if (lane != leader) continue;
                int h = (int)(((uint32_t)L * 2654435761u) >> 22) & (CL_HT - 1);
                bool done = false;
                for (int probe = 0; probe < 32; ++probe) {
                    const int old = atomicCAS(hkey + h, 0, L);
                    if (old == 0 || old == L) {
                        atomicAdd(hneg + h, sn);
                        atomicAdd(hpos + h, sp);
                        done = true;
                        break;
                    }
                    h = (h + 1) & (CL_HT - 1);
                }
                if (!done) {
                    if (sn) atomicAdd((unsigned long long *)(neg + L - 1), (unsigned long long)sn);
                    if (sp) atomicAdd((unsigned long long *)(pos + L - 1), (unsigned long long)sp);
                }
            }
        }
        y += dy;
        z += dz;
        if (y >= D.ny) {
            y -= D.ny;
            ++z;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CL_HT; i += CL_WG) {
        const int lab = hkey[i];
        if (lab <= 0) continue;
        if (hneg[i]) atomicAdd((unsigned long long *)(neg + lab - 1), (unsigned long long)hneg[i]);
        if (hpos[i]) atomicAdd((unsigned long long *)(pos + lab - 1), (unsigned long long)hpos[i]);
    }
}

__global__ __launch_bounds__(CL_WG) void k_cls_decide(const int64_t *nk, int64_t cap, const int64_t *neg,
                                                      const int64_t *pos, int8_t *inside) {
    const int64_t k = min(*nk, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x)
        inside[i] = neg[i] > pos[i] ? 1 : (pos[i] > neg[i] ? 0 : -1);
}

}  // namespace
}  // namespace hk

using namespace hk;

extern "C" int hk_classify(const float *I, const int32_t *labels, int32_t nx, int32_t ny, int32_t nz,
                           uint32_t periodic_mask, const int64_t *n_clusters, int64_t *neg, int64_t *pos,
                           int8_t *inside, hipStream_t stream) {
    if (!I || !labels || !n_clusters || !neg || !pos || !inside) return HK_ERR_INVALID_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || periodic_mask > 7u) return HK_ERR_INVALID_ARG;
    const int64_t n = (int64_t)nx * ny * nz;
    if (n > INT32_MAX) return HK_ERR_TOO_LARGE;
    const int64_t cap = (n + 1) / 2;  // clusters a lattice can hold (Sec. 3 bound)
    Dims D{nx, ny, nz, periodic_mask};
    const int64_t rows = (int64_t)ny * nz;
    const int64_t groups = std::max<int64_t>(1, (rows + 4 * CL_ROWS - 1) / (4 * CL_ROWS));
    const int small = (int)std::min<int64_t>((cap + CL_WG - 1) / CL_WG, 4096);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_cls_zero, dim3(small), dim3(CL_WG), 0, stream, n_clusters, cap, neg, pos);
    hipLaunchKernelGGL(k_cls_count, dim3((unsigned)groups), dim3(CL_WG), 0, stream, I, labels, D, n_clusters, cap,
                       neg, pos);
    hipLaunchKernelGGL(k_cls_decide, dim3(small), dim3(CL_WG), 0, stream, n_clusters, cap, neg, pos, inside);
    return hipGetLastError() == hipSuccess ? HK_OK : HK_ERR_HIP;
}
