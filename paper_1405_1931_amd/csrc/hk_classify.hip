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
constexpr int CL_MAXG = 2048;     // at most this many workgroups (a multiple of 8)
constexpr int CL_HT = 1024;       // LDS hash slots per workgroup
constexpr int CL_CH = 2;          // 64-site chunks of a row in flight per wave

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

// Adds the border-pair counts a lane holds for its E sites (cluster lab[e],
// counts cn[e] / cp[e]) to the workgroup's LDS hash.  Each pass takes one
// cluster -- the first pending one of the lowest pending lane -- sums what
// every lane holds for it over all its sites, and lets one lane update the
// hash (or, when the probe run is full, the global counters).  The wave sum
// is taken bit plane by bit plane with ballots: a lane holds at most 6 pairs
// per site, so its sum has 5 bits.
template <int E>
__device__ __forceinline__ void wave_add(const int (&lab)[E], int (&cn)[E], int (&cp)[E], int lane,
                                         int32_t *hkey, int32_t *hneg, int32_t *hpos, int64_t *neg, int64_t *pos) {
    static_assert(6 * E < 32, "a lane's sum must fit five bits");
    for (;;) {
        int mine = 0;
        bool pend = false;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!pend && (cn[e] | cp[e]) != 0) {
                mine = lab[e];
                pend = true;
            }
        const uint64_t m = __ballot(pend);
        if (m == 0) break;
        const int leader = __builtin_ctzll(m);
        const int L = __builtin_amdgcn_readlane(mine, leader);
        int sn = 0, sp = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if ((cn[e] | cp[e]) != 0 && lab[e] == L) {
                sn += cn[e];
                sp += cp[e];
                cn[e] = 0;
                cp[e] = 0;
            }
        int tn = 0, tp = 0;
#pragma unroll
        for (int bit = 0; bit < 5; ++bit) {
            tn += __popcll(__ballot((sn >> bit) & 1)) << bit;
            tp += __popcll(__ballot((sp >> bit) & 1)) << bit;
        }
        if (lane != leader) continue;
        int h = (int)(((uint32_t)L * 2654435761u) >> 22) & (CL_HT - 1);
        bool done = false;
        for (int probe = 0; probe < 32; ++probe) {
            const int old = atomicCAS(hkey + h, 0, L);
            if (old == 0 || old == L) {
                atomicAdd(hneg + h, tn);
                atomicAdd(hpos + h, tp);
                done = true;
                break;
            }
            h = (h + 1) & (CL_HT - 1);
        }
        if (!done) {
            if (tn) atomicAdd((unsigned long long *)(neg + L - 1), (unsigned long long)tn);
            if (tp) atomicAdd((unsigned long long *)(pos + L - 1), (unsigned long long)tp);
        }
    }
}

// The neighbour rows of lattice row r = (z, y), as offsets from the row's
// first site rb (wave-uniform), and whether each exists.
struct RowNb {
    uint32_t rb;
    int32_t off[4];  // y - 1, y + 1, z - 1, z + 1
    bool has[4];
};

// Per-workgroup LDS hash of (cluster, negative count, positive count).
struct Hash {
    int32_t *key, *neg, *pos;
};

// One wave takes CL_CH consecutive 64-site chunks of an x row (lane = x
// within a chunk), so the site and each of its six neighbour rows are
// coalesced row reads and no site index is ever divided.  Every load is
// unconditional, so that all of them are in flight together: a missing
// neighbour (or a lane past the row's end) reads the centre site (or the
// row's first site) instead, and the neighbour rule is applied to the loaded
// values afterwards.  The proximity values are loaded at the same sites, only
// when the wave holds a border pair.
__device__ __forceinline__ void row_sites(const float *I, const int32_t *labels, const Dims &D, const RowNb &R,
                                          int lane, int k, Hash h, int64_t *neg, int64_t *pos) {
    const bool px = D.mask & 1u;
    for (int x0 = 0; x0 < D.nx; x0 += 64 * CL_CH) {
        int lab[CL_CH], nl[CL_CH][6];
        uint32_t ad[CL_CH][6];
        bool has[CL_CH][6];
#pragma unroll
        for (int c = 0; c < CL_CH; ++c) {
            const int x = x0 + 64 * c + lane;
            const bool in = x < D.nx;
            const uint32_t ctr = in ? R.rb + x : R.rb;
            const int xm = step(x, -1, D.nx, px), xp = step(x, 1, D.nx, px);
            has[c][0] = in && xm >= 0;
            has[c][1] = in && xp >= 0;
            ad[c][0] = has[c][0] ? R.rb + xm : ctr;
            ad[c][1] = has[c][1] ? R.rb + xp : ctr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                has[c][2 + q] = in && R.has[q];
                ad[c][2 + q] = has[c][2 + q] ? ctr + R.off[q] : ctr;
            }
            const int v = labels[ctr];
            lab[c] = in ? v : 0;
#pragma unroll
            for (int d = 0; d < 6; ++d) nl[c][d] = labels[ad[c][d]];
        }
        bool bp[CL_CH][6];
        bool any = false;
#pragma unroll
        for (int c = 0; c < CL_CH; ++c) {
            const bool cl = lab[c] > 0 && lab[c] <= k;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                bp[c][d] = cl && has[c][d] && nl[c][d] == 0;
                any |= bp[c][d];
            }
        }
        if (__ballot(any) == 0) continue;  // no border pair in these chunks
        float iv[CL_CH][6];
#pragma unroll
        for (int c = 0; c < CL_CH; ++c)
#pragma unroll
            for (int d = 0; d < 6; ++d) iv[c][d] = I[ad[c][d]];
        int cn[CL_CH], cp[CL_CH];
#pragma unroll
        for (int c = 0; c < CL_CH; ++c) {
            cn[c] = 0;
            cp[c] = 0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int sd = bp[c][d] ? side_of(iv[c][d]) : 0;
                cn[c] += sd < 0;
                cp[c] += sd > 0;
            }
        }
        wave_add<CL_CH>(lab, cn, cp, lane, h.key, h.neg, h.pos, neg, pos);
    }
}

// The same for rows whose length is a multiple of 4 sites with both arrays
// 16-byte aligned: a lane takes four consecutive sites with one 16-byte
// load per row, so 256 sites of a row need seven loads of labels (the row,
// its four neighbour rows, and the x neighbours of the lane's end sites)
// and seven of I, against 52 single-site loads.
__device__ __forceinline__ void row_quads(const float *I, const int32_t *labels, const Dims &D, const RowNb &R,
                                          int lane, int k, Hash h, int64_t *neg, int64_t *pos) {
    const bool px = D.mask & 1u;
    for (int x0 = 0; x0 < D.nx; x0 += 256) {
        const int xs = x0 + 4 * lane;  // the lane's first site; all four lie in the row when in
        const bool in = xs < D.nx;
        const uint32_t ctr = in ? R.rb + xs : R.rb;
        const int xl = step(xs, -1, D.nx, px), xr = step(xs + 3, 1, D.nx, px);
        const bool hl = in && xl >= 0, hr = in && xr >= 0;
        const uint32_t al = hl ? R.rb + xl : ctr, ar = hr ? R.rb + xr : ctr;
        bool hn[4];
        uint32_t an[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hn[q] = in && R.has[q];
            an[q] = hn[q] ? ctr + R.off[q] : ctr;
        }
        const int4 c4 = *reinterpret_cast<const int4 *>(labels + ctr);
        const int lft = labels[al], rgt = labels[ar];
        int4 n4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) n4[q] = *reinterpret_cast<const int4 *>(labels + an[q]);
        const int cl[4] = {in ? c4.x : 0, in ? c4.y : 0, in ? c4.z : 0, in ? c4.w : 0};
        bool bp[4][6];
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool isc = cl[j] > 0 && cl[j] <= k;
            // x - 1 and x + 1: inside the quad, or the loaded end neighbours
            bp[j][0] = isc && (j > 0 ? cl[j - 1] == 0 : (hl && lft == 0));
            bp[j][1] = isc && (j < 3 ? cl[j + 1] == 0 : (hr && rgt == 0));
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = j == 0 ? n4[q].x : j == 1 ? n4[q].y : j == 2 ? n4[q].z : n4[q].w;
                bp[j][2 + q] = isc && hn[q] && v == 0;
            }
#pragma unroll
            for (int d = 0; d < 6; ++d) any |= bp[j][d];
        }
        if (__ballot(any) == 0) continue;
        const float4 i4 = *reinterpret_cast<const float4 *>(I + ctr);
        const float il = I[al], ir = I[ar];
        float4 m4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) m4[q] = *reinterpret_cast<const float4 *>(I + an[q]);
        const float ic[4] = {i4.x, i4.y, i4.z, i4.w};
        int cn[4], cp[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float iv[6];
            iv[0] = j > 0 ? ic[j - 1] : il;
            iv[1] = j < 3 ? ic[j + 1] : ir;
#pragma unroll
            for (int q = 0; q < 4; ++q) iv[2 + q] = j == 0 ? m4[q].x : j == 1 ? m4[q].y : j == 2 ? m4[q].z : m4[q].w;
            cn[j] = 0;
            cp[j] = 0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int sd = bp[j][d] ? side_of(iv[d]) : 0;
                cn[j] += sd < 0;
                cp[j] += sd > 0;
            }
        }
        wave_add<4>(cl, cn, cp, lane, h.key, h.neg, h.pos, neg, pos);
    }
}

// Counts the border pairs of every cluster.  Workgroups are dealt to the
// eight XCDs in turn; they are renumbered so that each XCD takes one
// contiguous range of rows (whole z planes at a time), and the y and z
// neighbour rows a workgroup reads sit in its own XCD's L2.  A workgroup
// takes rpw consecutive rows r = (z, y); wave w takes rows w, w + 4, ...; y
// and z advance with a carry, so no row index is divided inside the loop.
// Few, long workgroups keep the global adds to a cluster that spans the
// lattice (the exterior) at two per workgroup.
template <bool QUADS>
__global__ __launch_bounds__(CL_WG) void k_cls_count(const float *I, const int32_t *labels, Dims D, int rpw,
                                                     const int64_t *nk, int64_t cap, int64_t *neg, int64_t *pos) {
    __shared__ int32_t hkey[CL_HT];
    __shared__ int32_t hneg[CL_HT];
    __shared__ int32_t hpos[CL_HT];
    for (int i = threadIdx.x; i < CL_HT; i += CL_WG) {
        hkey[i] = 0;
        hneg[i] = 0;
        hpos[i] = 0;
    }
    __syncthreads();
    const Hash h{hkey, hneg, hpos};
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwv = CL_WG / 64;
    const int k = (int)min(*nk, cap);
    const bool py = D.mask & 2u, pz = D.mask & 4u;
    int b = blockIdx.x;
    const int G = gridDim.x;
    if ((G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
    const int rows = D.ny * D.nz;
    const int64_t first = (int64_t)b * rpw;
    const int rend = (int)min((int64_t)rows, first + rpw);
    int r = (int)(first + wv);
    int z = r / D.ny, y = r - z * D.ny;
    const int dz = nwv / D.ny, dy = nwv - dz * D.ny;
    const int64_t plane = (int64_t)D.ny * D.nx;
    for (; r < rend; r += nwv) {
        RowNb R;
        R.rb = (uint32_t)r * (uint32_t)D.nx;  // < 2^31 sites
        const int ym = step(y, -1, D.ny, py), yp = step(y, 1, D.ny, py);
        const int zm = step(z, -1, D.nz, pz), zp = step(z, 1, D.nz, pz);
        R.has[0] = ym >= 0;
        R.has[1] = yp >= 0;
        R.has[2] = zm >= 0;
        R.has[3] = zp >= 0;
        R.off[0] = (ym - y) * D.nx;
        R.off[1] = (yp - y) * D.nx;
        R.off[2] = (int32_t)((zm - z) * plane);
        R.off[3] = (int32_t)((zp - z) * plane);
        if (QUADS)
            row_quads(I, labels, D, R, lane, k, h, neg, pos);
        else
            row_sites(I, labels, D, R, lane, k, h, neg, pos);
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
    // rows per workgroup: at least 32, a multiple of the 4 waves, and enough
    // that the grid stays within CL_MAXG workgroups
    int64_t rpw = std::max<int64_t>(32, (rows + CL_MAXG - 1) / CL_MAXG);
    rpw = (rpw + 3) & ~int64_t(3);
    // padded to a multiple of 8 so that the XCD renumbering applies; the
    // extra workgroups find no row
    const int64_t groups = (std::max<int64_t>(1, (rows + rpw - 1) / rpw) + 7) & ~int64_t(7);
    const int small = (int)std::min<int64_t>((cap + CL_WG - 1) / CL_WG, 4096);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_cls_zero, dim3(small), dim3(CL_WG), 0, stream, n_clusters, cap, neg, pos);
    // four sites per lane when every row starts 16-byte aligned
    const bool quads = nx % 4 == 0 && (((uintptr_t)I | (uintptr_t)labels) & 15u) == 0;
    if (quads)
        hipLaunchKernelGGL(k_cls_count<true>, dim3((unsigned)groups), dim3(CL_WG), 0, stream, I, labels, D, (int)rpw,
                           n_clusters, cap, neg, pos);
    else
        hipLaunchKernelGGL(k_cls_count<false>, dim3((unsigned)groups), dim3(CL_WG), 0, stream, I, labels, D, (int)rpw,
                           n_clusters, cap, neg, pos);
    hipLaunchKernelGGL(k_cls_decide, dim3(small), dim3(CL_WG), 0, stream, n_clusters, cap, neg, pos, inside);
    return hipGetLastError() == hipSuccess ? HK_OK : HK_ERR_HIP;
}
