// Device-side data layout and per-brick phases of the GPU Hoshen-Kopelman path.
//
// The lattice is cut into bricks of 64 x BY x BZ sites.  One brick row (64
// consecutive x-sites of one (y, z)) is one 64-bit occupancy word, so runs of
// occupied sites along x are bit runs and a wavefront ballot over 64 sites
// produces a word directly.  Every phase below works on one brick (or one
// block of WG lattice rows) with a WG-thread workgroup; in the brick phases
// TPR threads share a row, each owning a SLICE-bit slice of it.  The
// single-lattice kernels launch one workgroup per item; the batched kernels
// launch one workgroup per item of every job of a batch.
//
// Phases (paper correspondence in brackets):
//   local   phi -> occupancy words (ballot per row);    [Sec. 2 condition]
//           rules 2/3 on x-runs inside a brick (LDS):   [Sec. 2 rules 1-3,
//           components that touch a face shared with     restricted to a brick]
//           another brick (or a periodic wrap) become
//           global nodes; the rest are finished clusters
//   merge   union of nodes across brick faces and       [Sec. 3 halo /
//           periodic wraps, lock-free CAS linking         periodic equivalences]
//           toward the node with the lowest site
//   roots   flatten node trees, accumulate cluster      [Sec. 3 list traversal
//           sizes at each root, mark root sites           to the lowest label]
//   rowsum / scanblk / rowpre: prefix count of roots    [Sec. 2 compaction to
//           over occupancy words in linear order          1..n]
//   write   component slot -> 1 + rank of its root,     [Sec. 2 final pass,
//           sizes from the root, labels of all sites      Sec. 5 sizes]
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace hk {

constexpr int WG = 512;               // threads per workgroup (8 wave64)
constexpr int NW = WG / 64;           // waves per workgroup
constexpr int TPR = 2;                // threads per brick row
constexpr int SLICE = 64 / TPR;       // bits of a row owned by one thread
constexpr int RMAX = WG / TPR;        // rows per brick at most (BY * BZ)
constexpr int MAXRUNS = 32 * RMAX;    // a 64-bit row holds at most 32 runs
constexpr int LPOS_BITS = RMAX <= 256 ? 14 : 15;  // bits of a brick-local site position row*64+x
static_assert(RMAX <= 512, "run ids, positions and sizes are packed for at most 512 rows");
static_assert(64 * RMAX <= (1 << 14), "brick sizes are accumulated as size << 16 in an int32");
// the roots phase: 512 threads over the nodes of ROOTS_MAX bricks (measured
// against 128 and 256: more nodes per workgroup keep more finds in flight)
constexpr int WG_NODES = 512;
// the merge phase: two waves per brick, sixteen bricks per CU in flight
constexpr int WG_MERGE = 128;
constexpr uint16_t NOSITE = 0xFFFF;   // face-table entry of an empty site
constexpr int GUARD = 1 << 22;        // bound on any retry/walk loop

// Fallback counters: each counts the times a bounded fast structure was
// full and the slower exact path took over (tests use them to show that a
// fallback ran; the results are the same either way).
constexpr int DBG_MERGE_DIRECT = 0;  // merge pairs united where found (LDS pair list full)
constexpr int DBG_ROOTS_DIRECT = 1;  // node sizes added to the root directly (LDS hash probes exhausted)
constexpr int DBG_EQUIV_AGAIN = 2;   // bricks whose equivalence list overflowed (overlaps united again)
constexpr int DBG_RUNS_GLOBAL = 3;   // bricks whose run slots did not fit the write phase's LDS
constexpr int DBG_N = 4;

// device-side check codes (sticky flag, never a fault)
constexpr int ERR_LOOP = 1;
constexpr int ERR_CAP = 2;
constexpr int ERR_FACE = 4;
constexpr int ERR_RANGE = 8;

struct Geo {
    // lattice
    int32_t nx, ny, nz;
    uint32_t mask;
    // bricks
    int32_t BY, BZ, lby, lbz, R;
    int32_t nbx, nby, nbz, nb;
    int32_t cap;      // node slots per brick
    int32_t fstride;  // x-face table entries per brick (2 R)
    int32_t rows;     // ny * nz lattice rows
    int32_t nblk;     // ceil(rows / WG)
    // division of a site index (below 2^31) by nx * ny and by nx: multiplier
    // and shift of the round-up method for 32-bit dividends (see fast_div)
    uint32_t dm_xy, dm_x;
    int32_t ds_xy, ds_x;
    // caller buffers
    const float *phi;  // the field (float32, or uint8 for PK_U8)
    int32_t tkey;      // order key of the predicate's threshold / value
    int32_t *labels;
    int64_t *n_clusters;
    int64_t *sizes;
    // workspace
    uint64_t *occ;    // [nb][R] occupancy words, brick-major
    uint64_t *root;   // [nb][R] bit set at the lowest site of every cluster
    int32_t *wpre;    // [nb][R] #cluster roots before this word, linear order
    uint16_t *face;   // [nb][fstride] node slot at each x-face site of each row
    int32_t *bcount;  // [nb] nodes used by each brick
    int32_t *npar;    // [nb*cap] node parent; at a root, -1 - the root's key (see g_find)
    int32_t *nkey;    // [nb*cap] linear index of the node's lowest site (incremental calls only)
    int32_t *nsize;   // [nb*cap] sites in the node; at a root, the cluster
    uint16_t *nlpos;  // [nb*cap] brick-local position row*64 + x of the key
    int32_t *nrootkey; // [nb*cap] key of the node's root (the linear index of its cluster's lowest site)
    int32_t *nrun;    // [nb] runs of each brick
    uint16_t *runlab; // [nb][runcap] component slot of every run of the brick
    uint32_t *icomp;  // [nb][icap] interior component: size << LPOS_BITS | key position
    int32_t *icount;  // [nb] interior components of each brick
    int32_t runcap;   // run slots per brick
    int32_t icap;     // interior component slots per brick
    int32_t *slab;    // [nb*cap] final label of each node's cluster
    uint16_t *rowo;   // [nb][R] id of the first run of each brick row
    int32_t *rowcnt;  // [rows] roots per lattice row
    int32_t *blksum;  // [nblk] roots per block of rows, then their prefix
    int32_t *err;     // sticky check flag
    uint32_t *dbg;    // [DBG_N] fallback counters (see DBG_*), or null
    // incremental relabelling of a field that changes little between calls:
    // 0 off; 1 label every brick and keep the copies below; 2 as 1, but a
    // brick whose occupancy words equal those of the previous call keeps its
    // local labelling (node, interior component, run and face tables)
    int32_t incr;
    int32_t *nsize0;    // [nb*cap] size of each node's brick-local component
    uint64_t *rootw0;   // [nb][R] root bits of each brick's interior components
    int64_t *nchanged;  // bricks labelled anew by the call, or null
    // droplet statistics (Sec. 5) gathered by the rank phase, where every
    // cluster's final size is at hand (hk_label_droplets; ds_part null: off)
    int64_t *ds_part;   // [ds_nbins + 2][DS_PARTS] partial bin counts, count, summed size
    double *ds_psum;    // [3][DS_PARTS] partial sums of R, R^2, R^3
    int64_t *ds_hist;   // [ds_nbins] out
    int64_t *ds_counts; // [2] out
    double *ds_sums;    // [3] out
    int64_t ds_min;     // clusters of fewer sites are left out
    double ds_rmax;     // histogram range [0, r_max)
    int32_t ds_nbins;   // 1 .. DS_MAXBINS
};

__host__ __device__ __forceinline__ int n_nodes(const Geo &g) { return g.nb * g.cap; }
__host__ __device__ __forceinline__ int64_t n_sites(const Geo &g) { return (int64_t)g.nx * g.ny * g.nz; }

struct Brick {
    int b, bx, by, bz;
    int x0, y0, z0;
    int ex, ey, ez;                    // extents (partial at the high ends)
    bool hxl, hxh, hyl, hyh, hzl, hzh; // face shared with another brick or a wrap
};

struct __align__(16) LdsBrick {
    uint64_t occ[RMAX];
    uint64_t rootw[RMAX];
    int32_t rowoff[RMAX + 1];
    int32_t wpre[RMAX];
    uint32_t bflag[MAXRUNS / 32];
    int32_t tmp[32];
    int32_t par[MAXRUNS];
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ void set_err(const Geo &g, int code) { atomicOr(g.err, code); }
__device__ __forceinline__ void count_dbg(const Geo &g, int i) {
    if (g.dbg) atomicAdd(g.dbg + i, 1u);
}

// Occupancy predicates.  PK_GT0 is the cluster condition phi > 0 of Sec. 2;
// the others let a caller label another set of sites (the capsule algorithm
// of Sec. 6 labels the sites whose proximity value equals the far-field
// value).  Values are the hk_predicate codes; PK_GT0 is internal.
constexpr int PK_GT = 0;   // float32 field > t
constexpr int PK_EQ = 1;   // float32 field == t
constexpr int PK_U8 = 2;   // uint8 field != 0
constexpr int PK_GT0 = 3;  // float32 field > 0
// value classes of the class test (bit k set: class k accepted): 7 positive
// denormal, 8 positive normal, 9 +infinity
constexpr int CLASS_POSITIVE = (1 << 7) | (1 << 8) | (1 << 9);

// An integer key that orders float bit patterns as IEEE orders the values:
// -|b| for negative values, b otherwise, so +0 and -0 share key 0 and
// denormals keep their place.  NaN patterns are excluded by the callers.
__host__ __device__ __forceinline__ int32_t order_key(uint32_t b) {
    return (b >> 31) ? -(int32_t)(b & 0x7fffffffu) : (int32_t)b;
}

// The predicate on a raw 32-bit load (float bits, or a zero-extended byte),
// decided on the bits so that no flush-to-zero mode can change it.
template <int PK>
__device__ __forceinline__ bool occupied_raw(uint32_t b, int32_t tkey) {
    if constexpr (PK == PK_GT0) {
        // positive denormal, normal or +inf (not NaN, not +-0, not negative):
        // one class test of the raw bits, which no denormal mode changes
        return __builtin_amdgcn_class(__uint_as_float(b), CLASS_POSITIVE);
    } else if constexpr (PK == PK_U8) {
        return b != 0u;
    } else {
        const bool num = (b & 0x7fffffffu) <= 0x7f800000u;  // not NaN
        if constexpr (PK == PK_GT) return num && order_key(b) > tkey;
        else return num && order_key(b) == tkey;
    }
}

// a raw value that no predicate accepts (a NaN pattern, or a zero byte)
template <int PK>
__device__ __forceinline__ constexpr uint32_t raw_empty() {
    return PK == PK_U8 ? 0u : 0x7fc00000u;
}

__device__ __forceinline__ uint64_t run_starts(uint64_t w) { return w & ~(w << 1); }

// bits 0..b inclusive
__device__ __forceinline__ uint64_t mask_le(int b) { return b >= 63 ? ~0ull : ((2ull << b) - 1ull); }

// set bits of x at positions 0..b, for 0 <= b <= 63 (one shift, no mask)
__device__ __forceinline__ int pop_le(uint64_t x, int b) { return __popcll(x << (63 - b)); }

// bits 0..b-1
__device__ __forceinline__ uint64_t mask_lt(int b) { return b <= 0 ? 0ull : (b >= 64 ? ~0ull : ((1ull << b) - 1ull)); }

// the SLICE bits of a row owned by slice q
__device__ __forceinline__ uint64_t slice_bits(int q) { return (~0ull >> (64 - SLICE)) << (SLICE * q); }

// length of the run of ones starting at bit s
__device__ __forceinline__ int run_len(uint64_t w, int s) {
    const uint64_t x = ~(w >> s);
    return x ? __builtin_ctzll(x) : 64;
}

__device__ __forceinline__ int lds_ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gl_st(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-uniform values (the row, its word, its run starts, its base address)
// are made scalar explicitly: the compiler cannot tell that threadIdx.x / 64
// is the same across a wave, and per-row arithmetic left in vector registers
// costs a full wave instruction each.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// the value of lane j (a constant or wave-uniform index), whatever the
// execution mask; the result is wave-uniform
__device__ __forceinline__ int lane_value(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
// the runs of the wave-uniform row word w that end below this lane (the
// index within the row of the run holding an occupied lane's site)
__device__ __forceinline__ int runs_ending_below(uint64_t w) {
    const uint64_t e = w & ~(w >> 1);
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(e >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)e, 0u));
}
__device__ __forceinline__ uint64_t lane_value64(uint64_t v, int j) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// inclusive prefix sum over the 64 lanes of a wave, with DPP moves: shifts
// by 1, 2, 4 and 8 lanes within each row of 16 lanes, then lane 15 of rows 0
// and 2 added to rows 1 and 3, then lane 31 to rows 2 and 3 (a lane whose
// source is outside the row or whose row is masked off adds 0)
__device__ __forceinline__ int wave_incl_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// exclusive prefix sum over the WG threads of the workgroup; all threads call
__device__ __forceinline__ int block_excl_scan(int v, int32_t *tmp, int *total) {
    const int lane = threadIdx.x & 63, w = wave_uniform(threadIdx.x >> 6);
    const int x = wave_incl_scan(v);
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int p = tmp[i];
        base += (i < w) ? p : 0;
        tot += p;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__device__ __forceinline__ int block_sum(int v, int32_t *tmp) {
    int t;
    (void)block_excl_scan(v, tmp, &t);
    return t;
}

__device__ __forceinline__ Brick brick_of(const Geo &g, int b) {
    Brick k;
    k.b = b;
    k.bx = b % g.nbx;
    const int q = b / g.nbx;
    k.by = q % g.nby;
    k.bz = q / g.nby;
    k.x0 = k.bx * 64;
    k.y0 = k.by * g.BY;
    k.z0 = k.bz * g.BZ;
    k.ex = min(64, g.nx - k.x0);
    k.ey = min(g.BY, g.ny - k.y0);
    k.ez = min(g.BZ, g.nz - k.z0);
    const bool wx = (g.mask & 1u) && g.nx >= 2;
    const bool wy = (g.mask & 2u) && g.ny >= 2;
    const bool wz = (g.mask & 4u) && g.nz >= 2;
    k.hxl = k.bx > 0 || wx;
    k.hxh = k.bx < g.nbx - 1 || wx;
    k.hyl = k.by > 0 || wy;
    k.hyh = k.by < g.nby - 1 || wy;
    k.hzl = k.bz > 0 || wz;
    k.hzh = k.bz < g.nbz - 1 || wz;
    return k;
}

// x-face table sections of one brick: the slot of the first run of each row
// (when it starts at x = 0), then of the last run (when it ends at the
// brick's last x)
__device__ __forceinline__ int f_xlo(const Geo &) { return 0; }
__device__ __forceinline__ int f_xhi(const Geo &g) { return g.R; }

// --------------------------------------------------------------------------
// union-find inside LDS (runs of one brick): link toward the smaller run id,
// so every component's root is its first run in brick raster order, whose
// start is the component's lowest site.
// --------------------------------------------------------------------------

__device__ __forceinline__ int l_find(int32_t *par, int x) {
    for (int i = 0; i < GUARD; ++i) {
        const int p = lds_ld(par + x);
        if (p == x) return x;
        const int gp = lds_ld(par + p);
        if (gp == p) return p;
        lds_st(par + x, gp);  // path halving; gp is an ancestor of x
        x = gp;
    }
    return x;
}

__device__ __forceinline__ void l_unite(const Geo &g, int32_t *par, int a, int b) {
    for (int i = 0; i < GUARD; ++i) {
        a = l_find(par, a);
        b = l_find(par, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(par + a, b);
        if (old == a) return;
        a = old;  // a had been linked meanwhile: carry on from its new parent
    }
    set_err(g, ERR_LOOP);
}

// --------------------------------------------------------------------------
// union-find over global nodes: a root is linked (CAS) below the root whose
// key (linear index of its lowest site) is smaller, so each cluster's final
// root is the node holding the cluster's lowest site.  A root's entry holds
// -1 - its key (keys are below 2^31 - 1, so the entry is negative) and any
// other entry its parent's index: a find learns the root's key with the
// load that shows it is a root, and a link is a CAS from -1 - key to the
// new parent.
//
// Parent reads may be served by the XCD's own cache and so be stale: a stale
// parent is still an ancestor (trees only ever merge), so a find on stale
// values only takes a longer path, and a stale root entry only makes the
// link's CAS fail.  Writes stay device-coherent: links are CAS on the true
// entry, and a failed CAS returns the true parent, from which the union
// carries on, so every retry climbs the true tree.
// --------------------------------------------------------------------------

__device__ __forceinline__ int nd_ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Roots of two nodes at once, with their keys: the two pointer chases
// advance in lockstep, so their loads are in flight together.  With HALVE
// the paths are halved: only non-root entries are rewritten, always to an
// ancestor.
template <bool HALVE>
__device__ __forceinline__ void g_find2(const Geo &g, int &x, int &kx, int &y, int &ky) {
    int32_t *par = g.npar;
    const int nn = n_nodes(g);
    bool dx = false, dy = false;
    kx = ky = 0;
    for (int i = 0; i < GUARD; ++i) {
        if (dx && dy) return;
        const int px = dx ? -1 : nd_ld(par + x);
        const int py = dy ? -1 : nd_ld(par + y);
        if (px >= nn || py >= nn) {
            set_err(g, ERR_RANGE);
            return;
        }
        const int gx = (dx || px < 0) ? -1 : nd_ld(par + px);
        const int gy = (dy || py < 0) ? -1 : nd_ld(par + py);
        if (gx >= nn || gy >= nn) {
            set_err(g, ERR_RANGE);
            return;
        }
        if (!dx) {
            if (px < 0) {
                kx = -1 - px;
                dx = true;
            } else if (gx < 0) {
                x = px;
                kx = -1 - gx;
                dx = true;
            } else {
                if (HALVE) gl_st(par + x, gx);
                x = gx;
            }
        }
        if (!dy) {
            if (py < 0) {
                ky = -1 - py;
                dy = true;
            } else if (gy < 0) {
                y = py;
                ky = -1 - gy;
                dy = true;
            } else {
                if (HALVE) gl_st(par + y, gy);
                y = gy;
            }
        }
    }
    set_err(g, ERR_LOOP);
}

__device__ __forceinline__ void g_unite(const Geo &g, int a, int b) {
    const int nn = n_nodes(g);
    if ((unsigned)a >= (unsigned)nn || (unsigned)b >= (unsigned)nn) {
        set_err(g, ERR_RANGE);
        return;
    }
    for (int i = 0; i < GUARD; ++i) {
        int ka, kb;
        g_find2<true>(g, a, ka, b, kb);
        if (a == b) return;
        if (ka < kb) {
            const int t = a, tk = ka;
            a = b;
            ka = kb;
            b = t;
            kb = tk;
        }
        const int old = atomicCAS(g.npar + a, -1 - ka, b);
        if (old == -1 - ka) return;
        if ((unsigned)old >= (unsigned)nn) {
            set_err(g, ERR_RANGE);
            return;
        }
        a = old;  // a was linked meanwhile: carry on from its true parent
    }
    set_err(g, ERR_LOOP);
}

// --------------------------------------------------------------------------
// occupancy of one brick, straight from phi: each wave takes a band of
// rows; lane x loads site x of U rows at once, and one ballot per row turns
// the 64 sites into the row's word, kept in LDS and stored for the relabel
// pass
// --------------------------------------------------------------------------

constexpr int OCC_U = 16;  // rows a wave has in flight at once

// this wave's band of brick rows: [r0, r1)
__device__ __forceinline__ void wave_band(const Geo &g, int *r0, int *r1) {
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int rpw = (g.R + NW - 1) / NW;
    *r0 = wv * rpw;
    *r1 = min(g.R, *r0 + rpw);
}

// lane x loads site x of rows base .. base+OCC_U-1 as raw bits (a value no
// predicate accepts outside the lattice).  Every partial product of an index
// is a site index below N <= 2^31 - 1, so 32-bit arithmetic is exact.  A
// batch of rows that lies wholly inside a full brick (the common case) needs
// no bounds checks and no lane masks; the others check each row and lane.
template <int PK>
__device__ __forceinline__ uint32_t load_raw(const Geo &g, uint32_t i) {
    if constexpr (PK == PK_U8)
        return reinterpret_cast<const uint8_t *>(g.phi)[i];
    else
        return __float_as_uint(g.phi[i]);
}

template <int PK>
__device__ __forceinline__ void fetch_rows(const Geo &g, const Brick &k, int base, int r1, uint32_t (&v)[OCC_U]) {
    const int lane = threadIdx.x & 63;
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    const bool full = k.ex == 64 && k.ey == g.BY && k.ez == g.BZ && base + OCC_U <= r1;
    if (full) {
#pragma unroll
        for (int j = 0; j < OCC_U; ++j) {
            const int r = base + j;
            const int yl = r & (g.BY - 1), zl = r >> g.lby;
            const uint32_t ri = ((uint32_t)(k.z0 + zl) * ny + (uint32_t)(k.y0 + yl)) * nx + (uint32_t)k.x0;
            v[j] = load_raw<PK>(g, ri + (uint32_t)lane);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < OCC_U; ++j) {
        const int r = base + j;
        const int yl = r & (g.BY - 1), zl = r >> g.lby;
        v[j] = raw_empty<PK>();
        if (r < r1 && yl < k.ey && zl < k.ez && lane < k.ex) {
            const uint32_t ri = ((uint32_t)(k.z0 + zl) * ny + (uint32_t)(k.y0 + yl)) * nx + (uint32_t)k.x0;
            v[j] = load_raw<PK>(g, ri + (uint32_t)lane);
        }
    }
}

// one ballot per row: the row's occupancy word, to LDS (the brick's words
// are copied out to HBM once the whole brick is in)
template <int PK>
__device__ __forceinline__ void ballot_rows(const Geo &g, int base, int r1, const uint32_t (&v)[OCC_U], LdsBrick &s) {
    const int lane = threadIdx.x & 63;
    // all the batch's ballots first, then one store region for lane 0
    uint64_t m[OCC_U];
#pragma unroll
    for (int j = 0; j < OCC_U; ++j) m[j] = __ballot(occupied_raw<PK>(v[j], g.tkey));
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < OCC_U; ++j)
            if (base + j < r1) s.occ[base + j] = m[j];
    }
}

// occupancy of a brick, OCC_U rows in flight per wave
template <int PK>
__device__ __forceinline__ void load_occupancy(const Geo &g, const Brick &k, LdsBrick &s) {
    int r0, r1;
    wave_band(g, &r0, &r1);
    for (int base = r0; base < r1; base += OCC_U) {
        uint32_t v[OCC_U];
        fetch_rows<PK>(g, k, base, r1, v);
        ballot_rows<PK>(g, base, r1, v, s);
    }
}

// --------------------------------------------------------------------------
// brick-local labelling (local phase)
//   in : s.occ[0..R)
//   out: s.rowoff; s.par: non-root run -> root run, root run -> -1 - size;
//        s.bflag: root runs touching a shared face; per thread, the number of
//        roots and boundary roots before the runs of its slice
// --------------------------------------------------------------------------

__device__ __forceinline__ bool bflag_get(const LdsBrick &s, int id) { return (s.bflag[id >> 5] >> (id & 31)) & 1u; }
__device__ __forceinline__ void bflag_set(LdsBrick &s, int id) { atomicOr(&s.bflag[id >> 5], 1u << (id & 31)); }

// The serial pass's rules, applied to the overlap segments of a row with its
// predecessor row rp that start in slice q: the first overlap to claim a run
// links it into the tree of the overlapping run of rp (rule 2, the label of
// the single labelled neighbour); every further overlap is an equivalence
// (rule 3), stored after the live runs in the par array as (a << 16 | b)
// while room lasts.
// The thread's work lies in its SLICE bits of the row, so the loop runs on
// 32-bit words: the run ids count the starts below the slice once, then
// the starts up to the segment within the slice.
__device__ __forceinline__ void link_rows(LdsBrick &s, int rp, uint64_t w, uint64_t st, int first, int q, int nruns) {
    const int sh = SLICE * q;
    const uint64_t wp = s.occ[rp];
    const uint64_t o = w & wp;
    uint32_t seg = (uint32_t)((o & ~(o << 1)) >> sh);
    if (!seg) return;
    const uint64_t stp = run_starts(wp);
    const int cbase = s.rowoff[rp] + __popcll(stp & mask_lt(sh)) - 1;
    const uint32_t st32 = (uint32_t)(st >> sh), stp32 = (uint32_t)(stp >> sh);
    while (seg) {
        const int bb = __builtin_ctz(seg);
        seg &= seg - 1;
        const uint32_t le = (2u << bb) - 1u;  // bits 0..bb (all 32 for bb = 31)
        const int a = first - 1 + __popc(st32 & le);
        // link to c's parent (c itself while c is unlinked): an ancestor of c
        // and an earlier run, which keeps the trees about half as deep
        const int c = lds_ld(s.par + cbase + __popc(stp32 & le));
        if (atomicCAS(s.par + a, a, c) != a) {
            const int e = atomicAdd(&s.tmp[20], 1);
            if (nruns + e < MAXRUNS) s.par[nruns + e] = (a << 16) | c;
        }
    }
}

// union of every overlap segment of the row with rp in slice q (fallback)
__device__ __forceinline__ void unite_rows(const Geo &g, LdsBrick &s, int rp, uint64_t w, uint64_t st, int offr, int q) {
    const uint64_t wp = s.occ[rp];
    const uint64_t o = w & wp;
    uint64_t seg = o & ~(o << 1) & slice_bits(q);
    const uint64_t stp = run_starts(wp);
    const int offp = s.rowoff[rp];
    while (seg) {
        const int bb = __builtin_ctzll(seg);
        seg &= seg - 1;
        l_unite(g, s.par, offr + pop_le(st, bb) - 1, offp + pop_le(stp, bb) - 1);
    }
}

// every run's entry set to its root in one pass: each run walks up to its
// root.  Every parent is an earlier run (links and unions point to the
// smaller index), so a walk ends; the entries other threads write meanwhile
// are roots of their runs, hence ancestors, and only shorten it.
__device__ __forceinline__ void walk_flatten(LdsBrick &s, int nruns) {
    for (int x = threadIdx.x; x < nruns; x += WG) {
        const int p = lds_ld(s.par + x);
        int r = p;
        int gp = lds_ld(s.par + r);
        for (int i = 0; gp != r && i < nruns; ++i) {  // at most x steps
            r = gp;
            gp = lds_ld(s.par + r);
        }
        lds_st(s.par + x, r);
    }
    __syncthreads();
}

struct CoreOut {
    int nruns;       // runs in the brick
    int btot, itot;  // boundary and interior components of the brick
    int bpre, ipre;  // boundary / interior components whose root run precedes this thread's slice
    uint32_t rbits;  // start bits of this thread's root runs, relative to its slice
};

__device__ __forceinline__ CoreOut brick_core(const Geo &g, const Brick &k, LdsBrick &s) {
    const int t = threadIdx.x, row = t / TPR, q = t % TPR;
    const int R = g.R;
    const bool live = row < R;
    const uint64_t w = live ? s.occ[row] : 0ull;
    const uint64_t st = run_starts(w);
    const uint64_t mine = st & slice_bits(q);  // run starts owned by this thread
    int total;
    const int off = block_excl_scan(q == 0 ? __popcll(st) : 0, s.tmp, &total);
    if (live && q == 0) s.rowoff[row] = off;
    if (t == 0) {
        s.rowoff[R] = total;
        s.tmp[20] = 0;  // equivalence count
    }
    if (t < MAXRUNS / 32) s.bflag[t] = 0u;
    for (int x = t; x < total; x += WG) s.par[x] = x;  // every run its own root
    __syncthreads();
    const int offr = live ? s.rowoff[row] : 0;
    // id of the first run starting in this slice
    const int first = offr + __popcll(st & mask_lt(SLICE * q));

    // rules 2/3 inside the brick against the row below (y-1) and the plane
    // below (z-1); runs of different rows only meet there
    const int yl = row & (g.BY - 1), zl = row >> g.lby;
    if (live && w) {
        if (yl > 0) link_rows(s, row - 1, w, st, first, q, total);
        if (zl > 0) link_rows(s, row - g.BY, w, st, first, q, total);
    }
    __syncthreads();
    const int ne = s.tmp[20];

    // equivalences: union of the trees, linking toward the smaller run, so
    // each component's root is its first run.  Every parent is an earlier
    // run, so the finds of the unions walk the unflattened trees as they
    // are (halving them); one flatten at the end costs less than one here
    // and another after.
    const int stored = min(ne, MAXRUNS - total);
    for (int e = t; e < stored; e += WG) {
        const int v = s.par[total + e];
        l_unite(g, s.par, v >> 16, v & 0xFFFF);
    }
    __syncthreads();
    if (stored < ne) {
        if (t == 0) count_dbg(g, DBG_EQUIV_AGAIN);
        // no room for every equivalence: unite all overlaps again (idempotent)
        if (live && w) {
            if (yl > 0) unite_rows(g, s, row - 1, w, st, offr, q);
            if (zl > 0) unite_rows(g, s, row - g.BY, w, st, offr, q);
        }
        __syncthreads();
    }
    walk_flatten(s, total);

    // component sizes in one pass: every run subtracts len << 16 from its
    // root's entry, so a root entry reads as its own index before the first
    // subtraction and negative after it, while any other entry holds its
    // root's index (non-negative, smaller than its own).  The same pass
    // flags the components touching a face shared with another brick (or a
    // wrap): every run of a y or z face row, the run at x = 0 and the last
    // run of a row when it reaches the brick's last x.  The start bits of
    // the slice's root runs are kept for the passes over roots only.
    uint32_t rbits = 0;
    {
        const bool frow = (k.hyl && yl == 0) || (k.hyh && yl == k.ey - 1) || (k.hzl && zl == 0) ||
                          (k.hzh && zl == k.ez - 1);
        // x-face runs by id: the row's first run when it starts at x = 0, its
        // last when it reaches the brick's last x (-1: none)
        const int xlo = k.hxl && (w & 1ull) ? offr : -1;
        const int xhi = k.hxh && ((w >> (k.ex - 1)) & 1ull) ? offr + __popcll(st) - 1 : -1;
        uint32_t m = (uint32_t)(mine >> (SLICE * q));
        int id = first;
        while (m) {
            const int b32 = __builtin_ctz(m);
            const int sb = b32 + SLICE * q;
            m &= m - 1;
            const int v = s.par[id];
            const int r = (v == id || v < 0) ? id : v;
            if (r == id) rbits |= 1u << b32;
            atomicAdd(&s.par[r], -(run_len(w, sb) << 16));
            if (frow || id == xlo || id == xhi) bflag_set(s, r);
            ++id;
        }
    }
    __syncthreads();

    // the slice's components: its root runs, and those flagged boundary.  The
    // flags of the slice's runs are bits first, first + 1, ... of s.bflag, and
    // only root runs are ever flagged.  Their prefix over the slices numbers
    // the components in raster order.
    uint32_t bw = 0;
    if (rbits) {
        const int wi = first >> 5, sh = first & 31;
        const uint64_t two = ((uint64_t)(wi + 1 < MAXRUNS / 32 ? s.bflag[wi + 1] : 0u) << 32) | s.bflag[wi];
        bw = (uint32_t)(two >> sh) & ((1u << __popcll(mine)) - 1u);  // a slice holds at most 16 runs
    }
    const int cb = __popc(bw), ci = __popc(rbits) - cb;
    int tot;
    const int pre = block_excl_scan((ci << 16) | cb, s.tmp, &tot);
    CoreOut out;
    out.nruns = total;
    out.btot = tot & 0xFFFF;
    out.itot = tot >> 16;
    out.bpre = pre & 0xFFFF;
    out.ipre = pre >> 16;
    out.rbits = rbits;
    return out;
}

// root run of a run after brick_core (root runs hold negative values)
__device__ __forceinline__ int root_of(const LdsBrick &s, int run) {
    const int v = s.par[run];
    return v < 0 ? run : v;
}


// --------------------------------------------------------------------------
// phase: local -- label the brick, create its nodes, its interior component
// table, the component slot of every run and the face tables
// --------------------------------------------------------------------------

// After the brick's occupancy is in s.occ: label it, write its nodes,
// interior components, run slots and face tables.
__device__ __forceinline__ void local_labels(const Geo &g, const Brick &k, int b, LdsBrick &s) {
    const int t = threadIdx.x, row = t / TPR;
    const int R = g.R;
    if (t < R) s.rootw[t] = 0ull;
    __syncthreads();
    if (g.incr == 2) {
        // the same words give the same local labelling: restore only what
        // the later phases modify (node parents and sizes, the root bits)
        const bool diff = t < R && g.occ[(int64_t)b * R + t] != s.occ[t];
        if (!__syncthreads_or(diff)) {
            const int bc = g.bcount[b];
            for (int c = t; c < bc; c += WG) {
                const int n = b * g.cap + c;
                g.npar[n] = -1 - g.nkey[n];
                g.nsize[n] = g.nsize0[n];
            }
            if (t < R) g.root[(int64_t)b * R + t] = g.rootw0[(int64_t)b * R + t];
            return;
        }
    }
    if (g.incr != 0 && t == 0 && g.nchanged) atomicAdd((unsigned long long *)g.nchanged, 1ull);
    if (t < R) g.occ[(int64_t)b * R + t] = s.occ[t];  // the words, for the later phases
    const CoreOut co = brick_core(g, k, s);

    // One pass over the root runs: boundary components (global nodes) take
    // slots 0..B-1 and interior ones B..C-1, both in raster order of their
    // root runs, and each root run's entry becomes -1 - slot.  Each slot's
    // record -- size << LPOS_BITS | key position -- is staged in LDS after
    // the runs when it fits (almost always: C <= runs, and the array holds
    // MAXRUNS entries), and written out by slot once all are known, one
    // coalesced pass: a node (position, size and the parent entry that holds
    // its key) or an interior entry (the record itself).  Otherwise the pass
    // writes each record where it finds it.
    const int btot = co.btot, itot = co.itot;
    const int ncomp = btot + itot;
    const bool staged = co.nruns + ncomp <= MAXRUNS;
    uint32_t *stage = reinterpret_cast<uint32_t *>(s.par + co.nruns);
    if (row < R) {
        int bi = co.bpre, ii = co.ipre;
        const uint64_t w = s.occ[row];
        const uint64_t st = run_starts(w);
        const int q = t % TPR, sh = SLICE * q;
        uint32_t m = co.rbits;  // root runs only
        const uint32_t st32 = (uint32_t)(st >> sh);
        // ids of the runs that start below this slice, minus one
        const int base = s.rowoff[row] + __popcll(st & mask_lt(sh)) - 1;
        const int lp0 = row * 64 + sh;  // key position of the slice's bit 0
        uint32_t rw = 0;                 // root bits of the slice's interior components
        if (staged) {
            while (m) {
                const int b32 = __builtin_ctz(m);
                m &= m - 1;
                const int id = base + __popc(st32 & ((2u << b32) - 1u));
                const int size = (id - s.par[id]) >> 16;  // see the size pass
                const bool bnd = bflag_get(s, id);
                const int c = bnd ? bi++ : btot + ii++;
                rw |= bnd ? 0u : 1u << b32;
                stage[c] = ((uint32_t)size << LPOS_BITS) | (uint32_t)(lp0 + b32);
                s.par[id] = -1 - c;
            }
        } else {
            const int yl = row & (g.BY - 1), zl = row >> g.lby;
            while (m) {
                const int b32 = __builtin_ctz(m);
                const int sb = b32 + sh;
                m &= m - 1;
                const int id = base + __popc(st32 & ((2u << b32) - 1u));
                const int size = (id - s.par[id]) >> 16;  // see the size pass
                if (bflag_get(s, id)) {
                    const int c = bi++;
                    if (c < g.cap) {
                        const int n = b * g.cap + c;
                        const int key = (k.x0 + sb) + g.nx * ((k.y0 + yl) + g.ny * (k.z0 + zl));
                        g.nlpos[n] = (uint16_t)(row * 64 + sb);
                        g.nsize[n] = size;
                        if (g.incr != 0) {
                            g.nsize0[n] = size;
                            g.nkey[n] = key;
                        }
                        g.npar[n] = -1 - key;
                    } else {
                        set_err(g, ERR_CAP);
                    }
                    s.par[id] = -1 - c;
                } else {
                    // interior component: a finished cluster, key and size kept
                    const int i = ii++;
                    rw |= 1u << b32;
                    if (i < g.icap)
                        g.icomp[(int64_t)b * g.icap + i] = ((uint32_t)size << LPOS_BITS) | (uint32_t)(row * 64 + sb);
                    else
                        set_err(g, ERR_CAP);
                    s.par[id] = -1 - (btot + i);
                }
            }
        }
        if (rw) atomicOr(reinterpret_cast<uint32_t *>(&s.rootw[row]) + q, rw);
    }
    __syncthreads();
    if (staged) {
        const uint32_t pmask = (1u << LPOS_BITS) - 1u;
        const int nbw = min(btot, g.cap);
        int32_t *npar = g.npar + b * g.cap;
        int32_t *nsize = g.nsize + b * g.cap;
        uint16_t *nlpos = g.nlpos + b * g.cap;
        for (int c = t; c < nbw; c += WG) {
            const uint32_t rec = stage[c];
            const int lp = (int)(rec & pmask), size = (int)(rec >> LPOS_BITS);
            const int r = lp >> 6;
            const int key = (k.x0 + (lp & 63)) + g.nx * ((k.y0 + (r & (g.BY - 1))) + g.ny * (k.z0 + (r >> g.lby)));
            nlpos[c] = (uint16_t)lp;
            nsize[c] = size;
            npar[c] = -1 - key;
            if (g.incr != 0) {
                g.nsize0[b * g.cap + c] = size;
                g.nkey[b * g.cap + c] = key;
            }
        }
        const int niw = min(itot, g.icap);
        uint32_t *icomp = g.icomp + (int64_t)b * g.icap;
        for (int i = t; i < niw; i += WG) icomp[i] = stage[btot + i];
        if (t == 0 && (btot > g.cap || itot > g.icap)) set_err(g, ERR_CAP);
    }
    __syncthreads();
    if (t == 0) {
        g.bcount[b] = min(btot, g.cap);
        g.icount[b] = min(itot, g.icap);
        g.nrun[b] = min(co.nruns, g.runcap);
    }
    if (t < R) {
        g.rowo[(int64_t)b * R + t] = (uint16_t)s.rowoff[t];
        g.root[(int64_t)b * R + t] = s.rootw[t];
        if (g.incr != 0) g.rootw0[(int64_t)b * R + t] = s.rootw[t];
    }

    // component slot of every run, for the final pass
    {
        // two slots per 32-bit store (runcap is a multiple of four)
        uint32_t *L2 = reinterpret_cast<uint32_t *>(g.runlab + (int64_t)b * g.runcap);
        const int nr = min(co.nruns, g.runcap);
        for (int i = t; 2 * i < nr; i += WG) {
            const uint32_t lo = (uint16_t)(-1 - s.par[root_of(s, 2 * i)]);
            const uint32_t hi = 2 * i + 1 < nr ? (uint16_t)(-1 - s.par[root_of(s, 2 * i + 1)]) : 0u;
            L2[i] = lo | (hi << 16);
        }
    }

    // x-face tables (the y and z faces are found from the words, run offsets
    // and run slots by the merge phase)
    uint16_t *F = g.face + (int64_t)b * g.fstride;
    if (t < R) {
        const int yl = t & (g.BY - 1), zl = t >> g.lby;
        if (yl < k.ey && zl < k.ez) {
            const uint64_t w = s.occ[t];
            if (k.hxl) {
                uint16_t e = NOSITE;
                if (w & 1ull) {
                    const int bidx = -1 - s.par[root_of(s, s.rowoff[t])];
                    if (bidx >= 0 && bidx < g.cap) e = (uint16_t)bidx; else set_err(g, ERR_FACE);
                }
                F[f_xlo(g) + t] = e;
            }
            if (k.hxh) {
                uint16_t e = NOSITE;
                if ((w >> (k.ex - 1)) & 1ull) {
                    const int bidx = -1 - s.par[root_of(s, s.rowoff[t + 1] - 1)];
                    if (bidx >= 0 && bidx < g.cap) e = (uint16_t)bidx; else set_err(g, ERR_FACE);
                }
                F[f_xhi(g) + t] = e;
            }
        }
    }
}

template <int PK = PK_GT0>
__device__ __forceinline__ void phase_local(const Geo &g, int b, LdsBrick &s) {
    const Brick k = brick_of(g, b);
    load_occupancy<PK>(g, k, s);
    local_labels(g, k, b, s);
}


// --------------------------------------------------------------------------
// phase: merge -- unite the nodes that meet across the brick's low x, y and
// z faces (the high faces are the low faces of the next bricks; wraps pair
// the first and the last brick of a periodic axis).
//
// x face: the x-face tables hold the slot of each row's first run (when it
// starts at x = 0) and last run (when it ends at the brick's last x); one
// row per lane.  A row whose predecessor in the same plane (y - 1) also has
// both face sites occupied is skipped: the two sites on each side are
// face-adjacent, so that row already joined the same two components.
// y and z faces: the face row of this brick and the face row across it are
// whole brick rows.  Their common occupied sites form segments, and each
// segment joins exactly one run of each row; the runs' slots come from the
// run tables at the rows' first-run offsets.  One face row per wave, one
// site per lane: the lane at a segment start looks up the two slots and
// drops its pair when the previous segment of the row had the same one.
// The pairs are collected in LDS and then united, spread evenly over the
// workgroup.
// --------------------------------------------------------------------------

constexpr int MERGE_CAP = 1024;  // pairs held in LDS; further pairs are united where found
constexpr int MERGE_F = 8;       // y/z face rows a wave takes at a time

struct MergeLds {
    int2 pair[MERGE_CAP];
    int count;
};

__device__ __forceinline__ void merge_push(const Geo &g, MergeLds &m, int na, int nc) {
    const int i = atomicAdd(&m.count, 1);
    if (i < MERGE_CAP) {
        m.pair[i] = make_int2(na, nc);
    } else {
        g_unite(g, na, nc);
        count_dbg(g, DBG_MERGE_DIRECT);
    }
}

__device__ __forceinline__ void phase_merge(const Geo &g, int b, MergeLds &m) {
    const Brick k = brick_of(g, b);
    const int lane = threadIdx.x & 63;
    const int wv = wave_uniform(threadIdx.x >> 6), nw = blockDim.x >> 6;
    if (threadIdx.x == 0) m.count = 0;
    __syncthreads();
    const int bxn = k.bx > 0 ? b - 1 : b + (g.nbx - 1);
    const int byn = k.by > 0 ? b - g.nbx : b + (g.nby - 1) * g.nbx;
    const int bzn = k.bz > 0 ? b - g.nbx * g.nby : b + (g.nbz - 1) * g.nbx * g.nby;
    const uint16_t *Fs = g.face + (int64_t)b * g.fstride + f_xlo(g);
    const uint16_t *Gs = g.face + (int64_t)bxn * g.fstride + f_xhi(g);

    // extents of the neighbours across the low y and z faces (a wrap pairs
    // the brick with the last brick of the axis, which may be partial)
    const int eyn = k.by > 0 ? g.BY : g.ny - (g.nby - 1) * g.BY;
    const int ezn = k.bz > 0 ? g.BZ : g.nz - (g.nbz - 1) * g.BZ;
    const int cy = k.hyl ? k.ez : 0, cz = k.hzl ? k.ey : 0;
    const uint64_t le = mask_le(lane);
    // Step `it` of a wave takes x-face chunk `it` (64 rows) and y/z face
    // group `it` (MERGE_F face rows); the loads of both that need nothing
    // else are issued together, then the run slots of the y/z segments.
    const int nxc = k.hxl ? (g.R + 63) >> 6 : 0;
    const int nyz = (cy + cz + MERGE_F - 1) / MERGE_F;
    for (int it = wv; it < max(nxc, nyz); it += nw) {
        // x face: one row per lane
        const int e = 64 * it + lane;
        const int yl = e & (g.BY - 1), zl = e >> g.lby;
        const bool xvalid = it < nxc && e < g.R && yl < k.ey && zl < k.ez;
        uint16_t fa = NOSITE, fc = NOSITE;
        if (xvalid) {
            fa = Fs[e];
            fc = Gs[e];
        }
        // y/z faces: lane j < MERGE_F loads the words and first-run offsets of face row f0 + j
        const int f0 = MERGE_F * it;
        uint64_t lwa = 0, lwb = 0;
        int loa = 0, lob = 0;
        {
            const int f = f0 + lane;
            if (lane < MERGE_F && f < cy + cz) {
                int ra, rb, bn;
                if (f < cy) {
                    bn = byn;
                    ra = g.BY * f;
                    rb = (eyn - 1) + g.BY * f;
                } else {
                    bn = bzn;
                    ra = f - cy;
                    rb = (f - cy) + g.BY * (ezn - 1);
                }
                lwa = g.occ[(int64_t)b * g.R + ra];
                lwb = g.occ[(int64_t)bn * g.R + rb];
                loa = g.rowo[(int64_t)b * g.R + ra];
                lob = g.rowo[(int64_t)bn * g.R + rb];
            }
        }
        if (it < nxc) {
            // A row whose predecessor in the same plane (y - 1, lane - 1) also
            // has both face sites occupied is skipped: it joins the same two
            // components (lane 0 of a chunk that starts inside a y row,
            // BY > 64, looks at the row before itself)
            const bool both = fa != NOSITE && fc != NOSITE;
            bool prev = __shfl_up((int)both, 1, 64) != 0;
            if (lane == 0) prev = xvalid && yl > 0 && Fs[e - 1] != NOSITE && Gs[e - 1] != NOSITE;
            if (both && !(yl > 0 && prev)) {
                if (fa < g.cap && fc < g.cap)
                    merge_push(g, m, b * g.cap + fa, bxn * g.cap + fc);
                else
                    set_err(g, ERR_FACE);
            }
        }
        if (f0 >= cy + cz) continue;
        // Consecutive face rows of one face are neighbours across the
        // face's other axis, so a lane at a segment start drops its pair
        // when the same site of the face row before had the same pair (a
        // cluster that crosses a face meets the same two components row
        // after row).
        int sa[MERGE_F], sb[MERGE_F];
        uint64_t sgj[MERGE_F];
#pragma unroll
        for (int j = 0; j < MERGE_F; ++j) {
            const uint64_t wa = lane_value64(lwa, j);
            const uint64_t wb = lane_value64(lwb, j);
            const int oa = lane_value(loa, j), ob = lane_value(lob, j);
            const uint64_t o = wa & wb;
            sgj[j] = o & ~(o << 1);  // segment starts
            sa[j] = sb[j] = -1;
            const int ia = oa + runs_ending_below(wa);
            const int ib = ob + runs_ending_below(wb);
            if ((sgj[j] >> lane) & 1ull) {
                const int f = f0 + j;
                const int bn = f < cy ? byn : bzn;
                sa[j] = g.runlab[(int64_t)b * g.runcap + min(ia, g.runcap - 1)];
                sb[j] = g.runlab[(int64_t)bn * g.runcap + min(ib, g.runcap - 1)];
            }
        }
        // the pair (slots a << 16 | b) of the segment that covers each
        // lane's site, per row: that of the last segment start at or below
        // the lane.  A segment start's previous segment is the one covering
        // the lane below it (a start's lower neighbour is not in the
        // overlap), one DPP wave shift away.
        int cp = -1;  // the pair covering this lane in the previous face row of the same face
#pragma unroll
        for (int j = 0; j < MERGE_F; ++j) {
            const int f = f0 + j;
            if (f >= cy + cz) break;
            const uint64_t sg = sgj[j];
            const uint64_t o = lane_value64(lwa, j) & lane_value64(lwb, j);
            const int pr = (int)(((uint32_t)sa[j] << 16) | ((uint32_t)sb[j] & 0xFFFFu));  // -1 off the starts
            const uint64_t upto = sg & le;  // starts at or below this lane
            const int cl = upto ? 63 - __clzll(upto) : lane;
            const int xp = __shfl(pr, cl, 64);
            const int pp = __builtin_amdgcn_update_dpp(-1, xp, 0x138, 0xf, 0xf, false);  // wave_shr:1
            if ((sg >> lane) & 1ull) {
                const bool first_of_face = f == 0 || f == cy;
                const bool same_row = pp == pr;
                const bool same_col = j > 0 && !first_of_face && cp == pr;
                if (!same_row && !same_col) {
                    const int bn = f < cy ? byn : bzn;
                    if (sa[j] < g.cap && sb[j] < g.cap)
                        merge_push(g, m, b * g.cap + sa[j], bn * g.cap + sb[j]);
                    else
                        set_err(g, ERR_FACE);
                }
            }
            cp = ((o >> lane) & 1ull) ? xp : -1;
        }
    }
    __syncthreads();
    const int n = min(m.count, MERGE_CAP);
    for (int i = threadIdx.x; i < n; i += blockDim.x) g_unite(g, m.pair[i].x, m.pair[i].y);
}

// --------------------------------------------------------------------------
// phase: roots -- find the root of every node of the brick; roots mark their
// key site in the root bitmap, every node records where its root's key site
// is, and non-roots add their size to the root.
//
// Sizes of clusters that span many bricks (the spanning cluster spans all of
// them) are first summed per brick in an LDS hash keyed by root node, then
// added to the root with one global atomic per (brick, root), instead of one
// per node.  The finds here only read: every node is found once, and halving
// stores cost more write traffic than they save the finds that follow (0.33
// against 0.43 ms at 1024^3; the merge's finds do halve, which shortens the
// trees these finds climb).  The root's key is kept in its own array, written
// only by the node's thread.
// --------------------------------------------------------------------------

constexpr int HT_BITS = 10;  // 1024 slots: 8 KB of LDS (with the bricks' root words 12 KB per workgroup)
constexpr int HT = 1 << HT_BITS;  // hash slots: keys in hash[0, HT), sums in hash[HT, 2 HT)
static_assert(2 * HT <= MAXRUNS, "the hash must fit in the run array of LdsBrick");

// Bricks b0 .. b0 + nbr - 1 share the LDS hash, so a root that many bricks
// reach (the spanning cluster's) receives one global add per group of bricks.
constexpr int ROOTS_MAX = 2;  // bricks one roots workgroup may take

// floor(v / d) for 0 <= v < 2^31 and 1 <= d < 2^31, from the multiplier m
// and shift l of the round-up method for 32-bit unsigned dividends:
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, and the quotient is
// (t + ((v - t) >> 1)) >> (l - 1) with t the high word of m v; d = 1 has
// l = 0 and is the identity.  The host forms m and l (magic_div in the API).
__device__ __forceinline__ uint32_t fast_div(uint32_t v, uint32_t m, int l) {
    if (l == 0) return v;
    const uint32_t t = __umulhi(m, v);
    return (t + ((v - t) >> 1)) >> (l - 1);
}

// word position (word index << 6 | bit) of the site whose linear index is key
__device__ __forceinline__ int64_t key_word_pos(const Geo &g, int key) {
    const uint32_t z = fast_div((uint32_t)key, g.dm_xy, g.ds_xy);
    const uint32_t rxy = (uint32_t)key - z * (uint32_t)(g.nx * g.ny);
    const uint32_t y = fast_div(rxy, g.dm_x, g.ds_x);
    const int x = (int)(rxy - y * (uint32_t)g.nx);
    const int bx = x >> 6, by = (int)y >> g.lby, bz = (int)z >> g.lbz;
    const int r = ((int)y & (g.BY - 1)) + g.BY * ((int)z & (g.BZ - 1));
    return (((int64_t)((bz * g.nby + by) * g.nbx + bx) * g.R + r) << 6) | (x & 63);
}

// rbits: LDS words of the workgroup's bricks (ROOTS_MAX * RMAX).  A root node
// sets its root bit in its own brick's words, and only the workgroup that
// takes a brick touches that brick's words in this phase, so the bits are
// gathered in LDS and merged into the words with plain loads and stores
// instead of one device-scope atomic per root.
//
// The nodes of all the workgroup's bricks form one index range, two nodes
// per thread and step; a node's own position and size are requested with
// its first parent load; the root's key, which the find returns, is kept
// for the rank phase, which finds the key site's word from it.
__device__ __forceinline__ void phase_roots(const Geo &g, int b0, int nbr, int32_t *hash, uint64_t *rbits) {
    int32_t *hkey = hash, *hval = hash + HT;
    const int nt = blockDim.x;
    for (int i = threadIdx.x; i < HT; i += nt) {
        hkey[i] = -1;
        hval[i] = 0;
    }
    const int nbh = min(nbr, g.nb - b0);  // bricks of the workgroup
    const int nw = nbh * g.R;              // their words
    for (int i = threadIdx.x; i < nw; i += nt) rbits[i] = 0ull;
    // node counts of the bricks: c[j] nodes before brick b0 + j
    int cpre[ROOTS_MAX + 1];
    cpre[0] = 0;
#pragma unroll
    for (int j = 0; j < ROOTS_MAX; ++j) cpre[j + 1] = cpre[j] + (j < nbh ? g.bcount[b0 + j] : 0);
    const int total = cpre[ROOTS_MAX];
    __syncthreads();
    for (int i0 = threadIdx.x; i0 < total; i0 += 2 * nt) {
        const bool two = i0 + nt < total;
        int nd[2], bj[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = u ? (two ? i0 + nt : i0) : i0;
            int j = 0;
#pragma unroll
            for (int q = 1; q < ROOTS_MAX; ++q) j += i >= cpre[q] ? 1 : 0;
            bj[u] = j;
            nd[u] = (b0 + j) * g.cap + (i - cpre[j]);
        }
        const int lp0 = g.nlpos[nd[0]], lp1 = g.nlpos[nd[1]];
        const int sz0 = g.nsize[nd[0]], sz1 = g.nsize[nd[1]];
        int r0 = nd[0], r1 = nd[1], k0, k1;
        g_find2<false>(g, r0, k0, r1, k1);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !two) break;
            const int n = nd[u], r = u ? r1 : r0, lr = u ? lp1 : lp0;
            g.nrootkey[n] = u ? k1 : k0;
            if (r == n) {
                if ((lr >> 6) < g.R)
                    atomicOr((unsigned long long *)(rbits + bj[u] * g.R + (lr >> 6)), 1ull << (lr & 63));
                else
                    set_err(g, ERR_RANGE);
            } else {
                const int add = u ? sz1 : sz0;
                int h = (int)(((uint32_t)r * 2654435761u) >> (32 - HT_BITS));
                bool done = false;
                for (int probe = 0; probe < 64; ++probe) {
                    const int old = atomicCAS(hkey + h, -1, r);
                    if (old == -1 || old == r) {
                        atomicAdd(hval + h, add);
                        done = true;
                        break;
                    }
                    h = (h + 1) & (HT - 1);
                }
                if (!done) {
                    atomicAdd(g.nsize + r, add);
                    count_dbg(g, DBG_ROOTS_DIRECT);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HT; i += nt) {
        const int r = hkey[i];
        if (r >= 0) atomicAdd(g.nsize + r, hval[i]);
    }
    uint64_t *gw = g.root + (int64_t)b0 * g.R;
    for (int i = threadIdx.x; i < nw; i += nt) {
        const uint64_t m = rbits[i];
        if (m) gw[i] |= m;
    }
}

// --------------------------------------------------------------------------
// phases: prefix count of root bits over words in linear order
// --------------------------------------------------------------------------

__device__ __forceinline__ int64_t word_base(const Geo &g, int row) {
    const int y = row % g.ny, z = row / g.ny;
    const int by = y >> g.lby, yl = y & (g.BY - 1);
    const int bz = z >> g.lbz, zl = z & (g.BZ - 1);
    return ((int64_t)(by + g.nby * bz) * g.nbx) * g.R + (yl + g.BY * zl);
}

__device__ __forceinline__ void phase_rowsum(const Geo &g, int blk, int32_t *tmp) {
    const int row = blk * WG + threadIdx.x;
    int c = 0;
    if (row < g.rows) {
        const int64_t w0 = word_base(g, row);
        for (int bx = 0; bx < g.nbx; ++bx) c += __popcll(g.root[w0 + (int64_t)bx * g.R]);
        g.rowcnt[row] = c;
    }
    const int s = block_sum(c, tmp);
    if (threadIdx.x == 0) g.blksum[blk] = s;
}

__device__ __forceinline__ void phase_scanblk(const Geo &g, int32_t *tmp) {
    int carry = 0;
    for (int base = 0; base < g.nblk; base += WG) {
        const int i = base + threadIdx.x;
        const int v = i < g.nblk ? g.blksum[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, tmp, &tot);
        if (i < g.nblk) g.blksum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *g.n_clusters = (int64_t)carry;
}

__device__ __forceinline__ void phase_rowpre(const Geo &g, int blk, int32_t *tmp) {
    const int row = blk * WG + threadIdx.x;
    const int v = row < g.rows ? g.rowcnt[row] : 0;
    int tot;
    const int ex = block_excl_scan(v, tmp, &tot);
    if (row < g.rows) {
        int run = g.blksum[blk] + ex;
        const int64_t w0 = word_base(g, row);
        for (int bx = 0; bx < g.nbx; ++bx) {
            const int64_t i = w0 + (int64_t)bx * g.R;
            g.wpre[i] = run;
            run += __popcll(g.root[i]);
        }
    }
}

// --------------------------------------------------------------------------
// droplet statistics (Sec. 5): a cluster of s sites as the radius of the
// sphere of the same volume, R = (3 s / (4 pi))^(1/3).  The histogram bin is
// decided on the size, not on a computed radius: R >= e <=> s >= (4 pi / 3)
// e^3, with the thresholds of the edges e_i = i * r_max / n_bins computed in
// double as c * (e * e * e), c = 4 pi / 3, so the bin counts are exact
// integers whatever kernel gathers them.  The sums of R^k carry rounding in
// the order the reduction takes.
// --------------------------------------------------------------------------

constexpr int DS_MAXBINS = 2048;  // histogram bins at most
constexpr int DS_PARTS = 256;     // partial accumulators the rank workgroups spread their adds over

constexpr int DS_TAB = 256;       // sizes below this take R, R^2 and their bin from a table

// R, R^2 and the bin of the sizes 0 .. DS_TAB - 1, computed as ds_add would
// (most clusters are small, and a cube root in double is the costly step)
struct DsTab {
    double r[DS_TAB], r2[DS_TAB];
    int32_t bin[DS_TAB];
};

// the bin of a size: the number of edges e_1 .. e_{n-1} whose threshold
// c * (e * e * e), e = i * w, is <= sd (the thresholds as ds_init stores them)
__device__ __forceinline__ int ds_bin_of(double sd, double w, int n_bins) {
    const double c = 4.0 * M_PI / 3.0;
    int lo = 0, hi = n_bins;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const double e = mid * w;
        if (c * (e * e * e) <= sd) lo = mid; else hi = mid;
    }
    return lo;
}

// T[i] = threshold of edge i, h[i] = 0, for i < n_bins, and the small-size
// table (all threads call; no barrier)
__device__ __forceinline__ void ds_init(double r_max, int n_bins, double *T, int32_t *h, DsTab *tab, int tid, int nt) {
    const double w = r_max / n_bins;
    const double c = 4.0 * M_PI / 3.0;
    for (int i = tid; i < n_bins; i += nt) {
        const double e = i * w;
        T[i] = c * (e * e * e);
        h[i] = 0;
    }
    for (int i = tid; i < DS_TAB; i += nt) {
        const double sd = (double)i;
        const double r = cbrt(sd * (3.0 / (4.0 * M_PI)));
        tab->r[i] = r;
        tab->r2[i] = r * r;
        tab->bin[i] = ds_bin_of(sd, w, n_bins);
    }
}

// per-thread sums of the clusters counted
struct DsAcc {
    int64_t cnt = 0, ssum = 0;
    double sr = 0.0, sr2 = 0.0, sr3 = 0.0;
};

// count one cluster of s sites (s >= min_size) into the LDS histogram h and acc
__device__ __forceinline__ void ds_add(DsAcc &a, const double *T, int32_t *h, const DsTab *tab, int n_bins,
                                       int64_t min_size, int64_t s) {
    if (s < min_size) return;
    const double sd = (double)s;
    const double v = sd * (3.0 / (4.0 * M_PI));
    int lo;
    double r, r2;
    if (s >= 0 && s < DS_TAB) {
        lo = tab->bin[s];
        r = tab->r[s];
        r2 = tab->r2[s];
    } else {
        // T[lo] <= s < T[hi]
        lo = 0;
        int hi = n_bins;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (T[mid] <= sd) lo = mid; else hi = mid;
        }
        r = cbrt(v);
        r2 = r * r;
    }
    atomicAdd(&h[lo], 1);
    ++a.cnt;
    a.ssum += s;
    a.sr += r;
    a.sr2 += r2;
    a.sr3 += v;
}

constexpr int WG_RANK = 512;

// LDS of a rank workgroup that gathers the statistics
struct DsLds {
    double T[DS_MAXBINS];          // edge thresholds
    int32_t h[DS_MAXBINS];         // the workgroup's bin counts
    DsTab tab;                     // small sizes
    double red[5][WG_RANK / 64];   // per-wave sums
};

// a 64-bit value moved by one DPP step, as two 32-bit halves (a lane with
// no source, or in a masked-off row, gets 0)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_mov64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t bits64(int64_t x) { return (uint64_t)x; }
__device__ __forceinline__ uint64_t bits64(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ void from_bits64(uint64_t u, int64_t *x) { *x = (int64_t)u; }
__device__ __forceinline__ void from_bits64(uint64_t u, double *x) { *x = __longlong_as_double((long long)u); }

// the sum of x (int64 or double) over the wave's 64 lanes (all active), by
// the steps of wave_incl_scan: lane 63 ends with the total
template <class T>
__device__ __forceinline__ T wave_total64(T x) {
    T y;
    from_bits64(dpp_mov64<0x111, 0xf>(bits64(x)), &y); x += y;  // row_shr:1
    from_bits64(dpp_mov64<0x112, 0xf>(bits64(x)), &y); x += y;  // row_shr:2
    from_bits64(dpp_mov64<0x114, 0xf>(bits64(x)), &y); x += y;  // row_shr:4
    from_bits64(dpp_mov64<0x118, 0xf>(bits64(x)), &y); x += y;  // row_shr:8
    from_bits64(dpp_mov64<0x142, 0xa>(bits64(x)), &y); x += y;  // row_bcast:15
    from_bits64(dpp_mov64<0x143, 0xc>(bits64(x)), &y); x += y;  // row_bcast:31
    from_bits64(lane_value64(bits64(x), 63), &y);
    return y;
}

// the workgroup's counts and sums into partial accumulator blockIdx % DS_PARTS
// (all threads call; a workgroup that counted nothing adds nothing)
__device__ __forceinline__ void ds_flush(const Geo &g, const DsAcc &a, DsLds *dl) {
    if (!__syncthreads_or(a.cnt != 0)) return;
    const double v[5] = {(double)wave_total64(a.cnt), (double)wave_total64(a.ssum), wave_total64(a.sr),
                         wave_total64(a.sr2), wave_total64(a.sr3)};  // counts below 2^53: exact
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k) dl->red[k][w] = v[k];
    __syncthreads();
    const int p = blockIdx.x % DS_PARTS;
    for (int i = threadIdx.x; i < g.ds_nbins; i += blockDim.x)
        if (dl->h[i]) atomicAdd((unsigned long long *)(g.ds_part + (int64_t)i * DS_PARTS + p), (unsigned long long)dl->h[i]);
    if (threadIdx.x < 5) {
        const int k = threadIdx.x;
        double t = 0.0;
        for (int i = 0; i < WG_RANK / 64; ++i) t += dl->red[k][i];
        if (k < 2) {
            if (t > 0.0)
                atomicAdd((unsigned long long *)(g.ds_part + (int64_t)(g.ds_nbins + k) * DS_PARTS + p), (unsigned long long)t);
        } else if (t != 0.0) {
            atomicAdd(g.ds_psum + (k - 2) * DS_PARTS + p, t);
        }
    }
}

// the droplet statistics' partial accumulators cleared by workgroup blk of nblk
__device__ __forceinline__ void ds_clear(const Geo &g, int blk, int nblk) {
    const int64_t n = (int64_t)DS_PARTS * (g.ds_nbins + 2);
    for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < n; i += (int64_t)nblk * blockDim.x) g.ds_part[i] = 0;
    for (int i = blk * blockDim.x + threadIdx.x; i < 3 * DS_PARTS; i += nblk * blockDim.x) g.ds_psum[i] = 0.0;
}

// --------------------------------------------------------------------------
// phase: rank -- the final label of every node's cluster: 1 + the rank of the
// cluster's key site (its lowest site, found by the roots phase) among all
// key sites in linear order, from the root bit words and the per-word
// prefixes (the key site's word comes from the root's key, which the roots
// phase kept for every node).  The node that holds its cluster's key site (the root) also
// writes the cluster's size.  Each thread takes RANK_U nodes at a time and
// issues all their first loads, then all their dependent word loads, so one
// brick costs two memory round trips.  Interior components are ranked by the
// write phase from the brick's own words.
// --------------------------------------------------------------------------

constexpr int RANK_U = 4;

// Workgroups are dispatched to the eight XCDs in turn (workgroup i runs on XCD
// i % 8).  This mapping hands all nbx bricks of a brick-row (one (by, bz)) to
// the workgroups of one XCD, so that the partial cache lines which the bricks
// of a brick-row write to one output range (the sizes of clusters whose key
// sites share lattice rows) meet in that XCD's L2.  The grid is
// xcd_grid(g) workgroups; the surplus ones get -1.
constexpr int NXCD = 8;
__host__ __device__ __forceinline__ int64_t xcd_grid(const Geo &g) {
    const int64_t q = (int64_t)g.nby * g.nbz;
    return (int64_t)NXCD * g.nbx * ((q + NXCD - 1) / NXCD);
}
__device__ __forceinline__ int xcd_brick(const Geo &g, int i) {
    const int x = i % NXCD, j = i / NXCD;
    const int q = x + NXCD * (j / g.nbx), bx = j % g.nbx;
    return q < g.nby * g.nbz ? q * g.nbx + bx : -1;
}

// the same mapping over groups of RANK_BRICKS consecutive bricks of a
// brick-row: workgroup i takes the group's first brick (or -1)
constexpr int RANK_BRICKS = 2;
__host__ __device__ __forceinline__ int64_t xcd_grid_rank(const Geo &g) {
    const int64_t q = (int64_t)g.nby * g.nbz;
    return (int64_t)NXCD * ((g.nbx + RANK_BRICKS - 1) / RANK_BRICKS) * ((q + NXCD - 1) / NXCD);
}
__device__ __forceinline__ int xcd_brick_rank(const Geo &g, int i) {
    const int ng = (g.nbx + RANK_BRICKS - 1) / RANK_BRICKS;
    const int x = i % NXCD, j = i / NXCD;
    const int q = x + NXCD * (j / ng), bx = RANK_BRICKS * (j % ng);
    return q < g.nby * g.nbz ? q * g.nbx + bx : -1;
}

// Bricks b0 .. b0 + nbr - 1 (consecutive bricks of one brick-row) form one
// node range: each thread takes up to RANK_U nodes at a time, issues their
// loads together, then their dependent word loads.  With STATS the
// workgroup then gathers the droplet statistics of the clusters whose key
// site lies in its bricks: the root nodes' and the interior components'.
template <bool STATS = false>
__device__ __forceinline__ void phase_rank(const Geo &g, int b0, int nbr, DsLds *dl = nullptr) {
    const int64_t kmax = (n_sites(g) + 1) / 2;
    const int64_t words = (int64_t)g.nb * g.R;
    const int nbh = min(nbr, g.nb - b0);
    const int bc0 = g.bcount[b0];
    const int total = bc0 + (nbh > 1 ? g.bcount[b0 + 1] : 0);
    if constexpr (STATS) ds_init(g.ds_rmax, g.ds_nbins, dl->T, dl->h, &dl->tab, threadIdx.x, WG_RANK);
    for (int c0 = threadIdx.x; c0 < total; c0 += RANK_U * WG_RANK) {
        int n[RANK_U], key[RANK_U], lp[RANK_U];
        int64_t wb[RANK_U];
        int32_t sz[RANK_U];
#pragma unroll
        for (int u = 0; u < RANK_U; ++u) {
            const int c = c0 + u * WG_RANK;
            const int j = c < bc0 ? 0 : 1;
            n[u] = (b0 + j) * g.cap + (c - (j ? bc0 : 0));
            wb[u] = (int64_t)(b0 + j) * g.R;
            key[u] = 0;
            lp[u] = 0;
            sz[u] = 0;
            if (c >= total) continue;
            key[u] = g.nrootkey[n[u]];
            lp[u] = g.nlpos[n[u]];
            sz[u] = g.nsize[n[u]];
        }
        int64_t wi[RANK_U];
        int bit[RANK_U];
        bool own[RANK_U];
        uint64_t rw[RANK_U];
        int wp[RANK_U];
#pragma unroll
        for (int u = 0; u < RANK_U; ++u) {
            const int c = c0 + u * WG_RANK;
            wi[u] = -1;
            bit[u] = 0;
            own[u] = false;
            if (c < total) {
                const int64_t pos = key_word_pos(g, key[u]);
                wi[u] = pos >> 6;
                bit[u] = (int)(pos & 63);
                // the node holds its cluster's key site: it is the root
                own[u] = wi[u] == wb[u] + min(lp[u] >> 6, g.R - 1) && bit[u] == (lp[u] & 63);
            }
            const bool ok = wi[u] >= 0 && wi[u] < words;
            rw[u] = ok ? g.root[wi[u]] : 0ull;
            wp[u] = ok ? g.wpre[wi[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < RANK_U; ++u) {
            const int c = c0 + u * WG_RANK;
            if (c >= total) break;
            if (wi[u] < 0 || wi[u] >= words) {
                set_err(g, ERR_RANGE);
                g.slab[n[u]] = 0;
                continue;
            }
            const int rank = wp[u] + __popcll(rw[u] & mask_lt(bit[u]));
            g.slab[n[u]] = rank + 1;
            if (g.sizes && own[u]) {
                if (rank >= 0 && (int64_t)rank < kmax)
                    g.sizes[rank] = (int64_t)sz[u];
                else
                    set_err(g, ERR_RANGE);
            }
        }
    }
    if constexpr (STATS) {
        // a cluster's key site lies in its root node (the root carries the
        // smallest key), so the node clusters are the roots, and their entries
        // still hold -1 - key; the interior components are finished clusters
        // (the thresholds were set before the rank loop; one barrier orders them)
        __syncthreads();
        DsAcc acc;
        for (int j = 0; j < nbh; ++j) {
            const int b = b0 + j;
            const int nn = g.bcount[b], ni = g.icount[b];
            const uint32_t *ic = g.icomp + (int64_t)b * g.icap;
            for (int c = threadIdx.x; c < max(nn, ni); c += WG_RANK) {
                // a node's entry and size and an interior record, loaded together
                const int n = b * g.cap + c;
                const int par = c < nn ? g.npar[n] : 0;
                const int sz = c < nn ? g.nsize[n] : 0;
                const uint32_t rec = c < ni ? ic[c] : 0u;
                if (par < 0) ds_add(acc, dl->T, dl->h, &dl->tab, g.ds_nbins, g.ds_min, (int64_t)sz);
                if (c < ni) ds_add(acc, dl->T, dl->h, &dl->tab, g.ds_nbins, g.ds_min, (int64_t)(rec >> LPOS_BITS));
            }
        }
        ds_flush(g, acc, dl);
    }
}

// --------------------------------------------------------------------------
// phase: write -- every site takes the label of its run's component slot.
// The brick's words, slot labels and run slots are loaded together (the run
// slots to s.par[nc, nc + nr) when they fit, else they are read from global
// memory per site), then the run offsets of the rows are counted.
// --------------------------------------------------------------------------

// a copy of a wave-uniform value in a vector register, so that the
// arithmetic on it runs on the vector pipe
__device__ __forceinline__ uint32_t vgpr_copy(uint32_t x) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

// Expand run labels to sites, one lattice row per wave and one site per
// lane.  The two forms are kept apart so that the common one (run table in
// LDS) has no global load in its loop: loads and stores share one
// outstanding-memory counter, and a load in the loop body makes every row
// wait for all earlier label stores to drain.  The common form is bound by
// scalar issue, so it has no per-row branch on the lanes (every lane looks
// up a slot, clamped into the table, and the empty sites discard it) and
// forms the row address on the vector pipe.
// v in the lanes whose bit of the wave-uniform mask m is set, else 0
__device__ __forceinline__ int select_by_mask(uint64_t m, int v) {
    int r;
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(m));
    return r;
}

template <bool RUNS_IN_LDS, bool FULL>
__device__ __forceinline__ void write_rows(const Geo &g, const Brick &k, const LdsBrick &s, int nc,
                                           const uint16_t *L) {
    const int lane = threadIdx.x & 63;
    // the lanes past the brick's last x have nothing to store; they leave
    // (lane 0 stays, so the wave-uniform reads below see a live lane)
    if (lane >= k.ex) return;
    const int wv = wave_uniform(threadIdx.x >> 6);
    const int runmax = g.runcap - 1;
    int32_t *const col = g.labels + k.x0 + lane;  // the lane's site in lattice row 0
    for (int r = wv; r < g.R; r += NW) {
        const int yl = r & (g.BY - 1), zl = r >> g.lby;
        if (!FULL && (yl >= k.ey || zl >= k.ez)) continue;
        const uint64_t wr = wave_uniform64(s.occ[r]);
        const int r0 = wave_uniform(s.rowoff[r]);  // id of the row's first run
        const int ends = runs_ending_below(wr);  // an occupied site's run within the row
        int lab;
        if constexpr (RUNS_IN_LDS) {
            // every lane looks up a slot (clamped into the table); the empty sites discard it
            const int slot = s.par[min(nc + r0 + ends, MAXRUNS - 1)];
            lab = select_by_mask(wr, s.par[min(max(slot, 0), MAXRUNS - 1)]);
        } else {
            lab = 0;
            if ((wr >> lane) & 1ull) {
                const int x = r0 + ends;
                const int slot = L[x < runmax ? x : runmax];
                lab = s.par[min(slot, MAXRUNS - 1)];
            }
        }
        // rows are below N <= 2^31 - 1: the row index fits 32 bits
        const uint32_t rowidx = vgpr_copy((uint32_t)((k.z0 + zl) * g.ny + (k.y0 + yl)));
        // the labels are written once and read by nobody in this call:
        // a streaming store, which does not keep the lines in L2
        __builtin_nontemporal_store(lab, col + (uint64_t)rowidx * (uint32_t)g.nx);
    }
}

template <bool RUNS_IN_LDS>
__device__ __forceinline__ void write_rows(const Geo &g, const Brick &k, const LdsBrick &s, int nc,
                                           const uint16_t *L) {
    if (k.ey == g.BY && k.ez == g.BZ)
        write_rows<RUNS_IN_LDS, true>(g, k, s, nc, L);
    else
        write_rows<RUNS_IN_LDS, false>(g, k, s, nc, L);
}

__device__ __forceinline__ void phase_write(const Geo &g, int b, LdsBrick &s) {
    const Brick k = brick_of(g, b);
    const int t = threadIdx.x;
    const int R = g.R;
    const int bc = g.bcount[b];
    const int nc = min(bc + g.icount[b], MAXRUNS);
    const int nr = g.nrun[b];
    const bool fit = nc + nr <= MAXRUNS;
    const uint16_t *L = g.runlab + (int64_t)b * g.runcap;
    if (t < R) {
        const int64_t i = (int64_t)b * R + t;
        s.occ[t] = g.occ[i];
        s.rootw[t] = g.root[i];
        s.wpre[t] = g.wpre[i];
        s.rowoff[t] = g.rowo[i];
    }
    // Every load is issued before the first wait: slot labels (nodes, from
    // the rank phase), raw interior entries and, when they fit, the run
    // slots four to a 64-bit word (runcap is a multiple of four).
    {
        for (int c0 = t; c0 < nc; c0 += 4 * WG) {
            int32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + u * WG;
                v[u] = c >= nc ? 0
                       : c < bc ? g.slab[b * g.cap + c] : (int32_t)g.icomp[(int64_t)b * g.icap + (c - bc)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + u * WG < nc) s.par[c0 + u * WG] = v[u];
        }
        if (fit) {
            const uint64_t *L4 = reinterpret_cast<const uint64_t *>(L);
            const int nq = (nr + 3) >> 2;
            for (int q0 = t; q0 < nq; q0 += 4 * WG) {
                uint64_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = q0 + u * WG < nq ? L4[q0 + u * WG] : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int id = 4 * (q0 + u * WG);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (id + j < nr) s.par[nc + id + j] = (int32_t)((v[u] >> (16 * j)) & 0xffffu);
                }
            }
        }
    }
    __syncthreads();

    // interior slots: rank of the key site from this brick's own words; the
    // slot writes its cluster's size
    const int64_t kmax = (n_sites(g) + 1) / 2;
    for (int c = bc + t; c < nc; c += WG) {
        const uint32_t u = (uint32_t)s.par[c];
        const int lp = (int)(u & ((1u << LPOS_BITS) - 1u));
        const int r = min(lp >> 6, R - 1);
        const int rank = s.wpre[r] + __popcll(s.rootw[r] & mask_lt(lp & 63));
        if (g.sizes) {
            if (rank >= 0 && (int64_t)rank < kmax)
                g.sizes[rank] = (int64_t)(u >> LPOS_BITS);
            else
                set_err(g, ERR_RANGE);
        }
        s.par[c] = rank + 1;
    }
    __syncthreads();

    if (fit) {
        write_rows<true>(g, k, s, nc, L);
    } else {
        if (threadIdx.x == 0) count_dbg(g, DBG_RUNS_GLOBAL);
        write_rows<false>(g, k, s, nc, L);
    }
}

// --------------------------------------------------------------------------
// batched launches: one kernel per phase covers the items of every job of
// the batch; workgroup w finds its job by a search over the per-phase item
// offsets.  The job table is written before the launches and never during
// them, so it is read through the constant address space: the compiler may
// keep or re-fetch its fields with scalar loads instead of treating every
// store of a phase as a possible write to them.
// --------------------------------------------------------------------------

constexpr int NPH = 8;  // local, merge, roots, rowsum, scanblk, rowpre, rank, write

typedef const __attribute__((address_space(4))) Geo ConstGeo;
typedef const __attribute__((address_space(4))) int32_t ConstI32;

struct GroupView {
    ConstGeo *jobs;
    ConstI32 *itoff;  // [NPH][njobs + 1] first item of each job within a phase
    int32_t njobs;
};

// job j and item i of workgroup `rel` in phase p: itoff[p][j] <= rel < itoff[p][j + 1]
// (every job has at least one item in every phase)
__device__ __forceinline__ const Geo &locate(const GroupView &v, int p, int rel, int *item) {
    ConstI32 *off = v.itoff + p * (v.njobs + 1);
    int lo = 0, hi = v.njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= rel) lo = mid; else hi = mid;
    }
    *item = rel - off[lo];
    return *(const Geo *)(v.jobs + lo);
}

}  // namespace hk
