// Device-side data layout and per-brick phases of the GPU Hoshen-Kopelman path.
//
// The lattice is cut into bricks of 64 x BY x BZ sites.  One brick row (64
// consecutive x-sites of one (y, z)) is one 64-bit occupancy word, so runs of
// occupied sites along x are bit runs and a wavefront ballot over 64 sites
// produces a word directly.  Every phase below works on one brick (or one
// block of 256 lattice rows) with a 256-thread workgroup; the single-lattice
// kernels launch one workgroup per item, the batched persistent kernel pulls
// the same items from a queue.
//
// Phases (paper correspondence in brackets):
//   pack    phi -> occupancy words                      [Sec. 2 condition]
//   local   union-find of x-runs inside a brick (LDS):  [Sec. 2 rules 1-3,
//           components that touch a face shared with     restricted to a brick]
//           another brick (or a periodic wrap) become
//           global nodes; the rest are final clusters
//   merge   union of nodes across brick faces and       [Sec. 3 halo /
//           periodic wraps, lock-free CAS linking         periodic equivalences]
//           toward the node with the lowest site
//   roots   flatten node trees, accumulate cluster      [Sec. 3 list traversal
//           sizes at each root, mark root sites           to the lowest label]
//   rowsum / scanblk / rowpre: prefix count of roots    [Sec. 2 compaction to
//           over occupancy words in linear order          1..n]
//   write   redo the brick labelling, map each          [Sec. 2 final pass,
//           component to 1 + rank of its root,            Sec. 5 sizes]
//           write labels and sizes
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int WG = 256;               // threads per workgroup (4 wave64)
constexpr int RMAX = 256;             // rows per brick at most (BY * BZ)
constexpr int MAXRUNS = 32 * RMAX;    // a 64-bit row holds at most 32 runs
constexpr uint16_t NOSITE = 0xFFFF;   // face-table entry of an empty site
constexpr int GUARD = 1 << 22;        // bound on any retry/walk loop

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
    int32_t fstride;  // face-table entries per brick
    int32_t rows;     // ny * nz lattice rows
    int32_t nblk;     // ceil(rows / WG)
    // caller buffers
    const float *phi;
    int32_t *labels;
    int64_t *n_clusters;
    int64_t *sizes;
    // workspace
    uint64_t *occ;    // [nb][R] occupancy words, brick-major
    uint64_t *root;   // [nb][R] bit set at the lowest site of every cluster
    int32_t *wpre;    // [nb][R] #cluster roots before this word, linear order
    uint16_t *face;   // [nb][fstride] node slot of each face site
    int32_t *bcount;  // [nb] nodes used by each brick
    int32_t *npar;    // [nb*cap] node parent
    int32_t *nkey;    // [nb*cap] linear index of the node's lowest site
    int32_t *nsize;   // [nb*cap] sites in the node; at a root, the cluster
    uint16_t *nlpos;  // [nb*cap] brick-local position row*64 + x of the key
    int32_t *rowcnt;  // [rows] roots per lattice row
    int32_t *blksum;  // [nblk] roots per block of rows, then their prefix
    int32_t *err;     // sticky check flag
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
    int32_t broff[RMAX + 1];
    int32_t wpre[RMAX];
    uint32_t bflag[MAXRUNS / 32];
    int32_t tmp[8];
    int32_t par[MAXRUNS];
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ void set_err(const Geo &g, int code) { atomicOr(g.err, code); }

// phi > 0 in IEEE single precision, decided on the bit pattern so that no
// flush-to-zero mode can change it: positive finite or +inf, not NaN, not +0.
__device__ __forceinline__ bool occupied(float v) {
    const int b = __float_as_int(v);
    return b > 0 && b <= 0x7f800000;
}

__device__ __forceinline__ uint64_t run_starts(uint64_t w) { return w & ~(w << 1); }

// bits 0..b inclusive
__device__ __forceinline__ uint64_t mask_le(int b) { return b >= 63 ? ~0ull : ((2ull << b) - 1ull); }

// bits 0..b-1
__device__ __forceinline__ uint64_t mask_lt(int b) { return b <= 0 ? 0ull : (b >= 64 ? ~0ull : ((1ull << b) - 1ull)); }

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
__device__ __forceinline__ int gl_ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gl_st(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive prefix sum over the 256 threads of the workgroup; all threads call
__device__ __forceinline__ int block_excl_scan(int v, int32_t *tmp, int *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) base += (i < w) ? tmp[i] : 0;
    const int tot = tmp[0] + tmp[1] + tmp[2] + tmp[3];
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

// face-table sections of one brick
__device__ __forceinline__ int f_xlo(const Geo &) { return 0; }
__device__ __forceinline__ int f_xhi(const Geo &g) { return g.R; }
__device__ __forceinline__ int f_ylo(const Geo &g) { return 2 * g.R; }
__device__ __forceinline__ int f_yhi(const Geo &g) { return 2 * g.R + 64 * g.BZ; }
__device__ __forceinline__ int f_zlo(const Geo &g) { return 2 * g.R + 128 * g.BZ; }
__device__ __forceinline__ int f_zhi(const Geo &g) { return 2 * g.R + 128 * g.BZ + 64 * g.BY; }

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

// walk to the root without writing (used once no more links happen)
__device__ __forceinline__ int l_root(int32_t *par, int x) {
    for (int i = 0; i < GUARD; ++i) {
        const int p = lds_ld(par + x);
        if (p == x) return x;
        x = p;
    }
    return x;
}

// --------------------------------------------------------------------------
// union-find over global nodes: a root is linked (CAS) below the root whose
// key (linear index of its lowest site) is smaller, so each cluster's final
// root is the node holding the cluster's lowest site.
// --------------------------------------------------------------------------

__device__ __forceinline__ int g_find(const Geo &g, int x) {
    int32_t *par = g.npar;
    const int nn = n_nodes(g);
    for (int i = 0; i < GUARD; ++i) {
        const int p = gl_ld(par + x);
        if (p == x) return x;
        if ((unsigned)p >= (unsigned)nn) {
            set_err(g, ERR_RANGE);
            return x;
        }
        const int gp = gl_ld(par + p);
        if (gp == p) return p;
        if ((unsigned)gp >= (unsigned)nn) {
            set_err(g, ERR_RANGE);
            return p;
        }
        gl_st(par + x, gp);  // path halving; only non-roots are rewritten
        x = gp;
    }
    set_err(g, ERR_LOOP);
    return x;
}

// walk to the root without writing: once no more links happen, each node's
// own entry is then written by exactly one thread (a halving store from a
// concurrent walk could otherwise overwrite a freshly flattened entry with
// an intermediate ancestor)
__device__ __forceinline__ int g_root(const Geo &g, int x) {
    const int nn = n_nodes(g);
    for (int i = 0; i < GUARD; ++i) {
        const int p = gl_ld(g.npar + x);
        if (p == x) return x;
        if ((unsigned)p >= (unsigned)nn) {
            set_err(g, ERR_RANGE);
            return x;
        }
        x = p;
    }
    set_err(g, ERR_LOOP);
    return x;
}

__device__ __forceinline__ void g_unite(const Geo &g, int a, int b) {
    const int nn = n_nodes(g);
    if ((unsigned)a >= (unsigned)nn || (unsigned)b >= (unsigned)nn) {
        set_err(g, ERR_RANGE);
        return;
    }
    for (int i = 0; i < GUARD; ++i) {
        a = g_find(g, a);
        b = g_find(g, b);
        if (a == b) return;
        if (g.nkey[a] < g.nkey[b]) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(g.npar + a, a, b) == a) return;
    }
    set_err(g, ERR_LOOP);
}

// --------------------------------------------------------------------------
// phase: pack phi into occupancy words (one workgroup per brick)
// --------------------------------------------------------------------------

__device__ __forceinline__ void phase_pack(const Geo &g, int b) {
    const Brick k = brick_of(g, b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int U = 16;
    for (int base = wv * 64; base < g.R; base += WG) {
        uint64_t mine = 0;
#pragma unroll
        for (int j0 = 0; j0 < 64; j0 += U) {
            float v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int r = base + j0 + j;
                const int yl = r & (g.BY - 1), zl = r >> g.lby;
                v[j] = 0.0f;
                if (r < g.R && yl < k.ey && zl < k.ez && lane < k.ex)
                    v[j] = g.phi[((int64_t)(k.z0 + zl) * g.ny + (k.y0 + yl)) * g.nx + k.x0 + lane];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const uint64_t m = __ballot(occupied(v[j]));
                if (lane == j0 + j) mine = m;
            }
        }
        if (base + lane < g.R) g.occ[(int64_t)b * g.R + base + lane] = mine;
    }
}

// --------------------------------------------------------------------------
// brick-local labelling shared by the local and write phases
//   in : s.occ[0..R)
//   out: s.rowoff, s.par (non-root run -> root run; root run -> -1 - size),
//        s.bflag (root runs touching a shared face), s.broff (prefix of such
//        roots per row, in run order)
// --------------------------------------------------------------------------

__device__ __forceinline__ void unite_rows(const Geo &g, LdsBrick &s, int r, int rp, uint64_t w, uint64_t st) {
    const uint64_t wp = s.occ[rp];
    const uint64_t o = w & wp;
    uint64_t seg = o & ~(o << 1);
    if (!seg) return;
    const uint64_t stp = run_starts(wp);
    const int offr = s.rowoff[r], offp = s.rowoff[rp];
    while (seg) {
        const int bb = __builtin_ctzll(seg);
        seg &= seg - 1;
        const uint64_t mk = mask_le(bb);
        const int a = offr + __popcll(st & mk) - 1;
        const int c = offp + __popcll(stp & mk) - 1;
        l_unite(g, s.par, a, c);
    }
}

__device__ __forceinline__ bool bflag_get(const LdsBrick &s, int id) { return (s.bflag[id >> 5] >> (id & 31)) & 1u; }
__device__ __forceinline__ void bflag_set(LdsBrick &s, int id) { atomicOr(&s.bflag[id >> 5], 1u << (id & 31)); }

__device__ __forceinline__ void brick_core(const Geo &g, const Brick &k, LdsBrick &s) {
    const int t = threadIdx.x;
    const int R = g.R;
    const uint64_t w = (t < R) ? s.occ[t] : 0ull;
    const uint64_t st = run_starts(w);
    const int nr = __popcll(st);
    int total;
    const int off = block_excl_scan(nr, s.tmp, &total);
    if (t < R) s.rowoff[t] = off;
    if (t == 0) s.rowoff[R] = total;
    s.bflag[t] = 0u;  // MAXRUNS / 32 == WG
    for (int j = 0; j < nr; ++j) s.par[off + j] = off + j;
    __syncthreads();

    // rules 2/3 inside the brick: runs overlapping in the row below (y-1)
    // and the plane below (z-1) are the same component
    const int yl = t & (g.BY - 1), zl = t >> g.lby;
    if (t < R && w) {
        if (yl > 0) unite_rows(g, s, t, t - 1, w, st);
        if (zl > 0) unite_rows(g, s, t, t - g.BY, w, st);
    }
    __syncthreads();

    for (int j = 0; j < nr; ++j) s.par[off + j] = l_root(s.par, off + j);
    __syncthreads();

    // components touching a face shared with another brick (or a wrap)
    if (t < R && w) {
        const bool frow = (k.hyl && yl == 0) || (k.hyh && yl == k.ey - 1) || (k.hzl && zl == 0) ||
                          (k.hzh && zl == k.ez - 1);
        if (frow) {
            for (int j = 0; j < nr; ++j) bflag_set(s, s.par[off + j]);
        } else {
            if (k.hxl && (w & 1ull)) bflag_set(s, s.par[off]);
            if (k.hxh && ((w >> (k.ex - 1)) & 1ull)) bflag_set(s, s.par[off + nr - 1]);
        }
    }
    __syncthreads();

    // component sizes, accumulated in the root entry as -1 - size
    {
        uint64_t m = st;
        int id = off;
        while (m) {
            const int sb = __builtin_ctzll(m);
            m &= m - 1;
            if (s.par[id] == id) s.par[id] = -1 - run_len(w, sb);
            ++id;
        }
    }
    __syncthreads();
    {
        uint64_t m = st;
        int id = off;
        while (m) {
            const int sb = __builtin_ctzll(m);
            m &= m - 1;
            const int p = s.par[id];
            if (p >= 0) atomicAdd(&s.par[p], -run_len(w, sb));
            ++id;
        }
    }
    __syncthreads();

    int bc = 0;
    for (int j = 0; j < nr; ++j) {
        const int id = off + j;
        bc += (s.par[id] < 0 && bflag_get(s, id)) ? 1 : 0;
    }
    int btot;
    const int boff = block_excl_scan(bc, s.tmp, &btot);
    if (t < R) s.broff[t] = boff;
    if (t == 0) s.broff[R] = btot;
    __syncthreads();
}

// root run of a run after brick_core (root runs hold negative values)
__device__ __forceinline__ int root_of(const LdsBrick &s, int run) {
    const int v = s.par[run];
    return v < 0 ? run : v;
}

// --------------------------------------------------------------------------
// phase: local -- label the brick, create its nodes and face tables
// --------------------------------------------------------------------------

__device__ __forceinline__ void phase_local(const Geo &g, int b, LdsBrick &s) {
    const Brick k = brick_of(g, b);
    const int t = threadIdx.x;
    const int R = g.R;
    if (t < R) s.occ[t] = g.occ[(int64_t)b * R + t];
    __syncthreads();
    brick_core(g, k, s);

    if (t < R) {
        const uint64_t w = s.occ[t];
        uint64_t m = run_starts(w);
        int id = s.rowoff[t];
        int bi = s.broff[t];
        const int yl = t & (g.BY - 1), zl = t >> g.lby;
        uint64_t rw = 0;
        while (m) {
            const int sb = __builtin_ctzll(m);
            m &= m - 1;
            const int v = s.par[id];
            if (v < 0) {
                if (bflag_get(s, id)) {
                    const int bidx = bi++;
                    if (bidx < g.cap) {
                        const int n = b * g.cap + bidx;
                        g.nkey[n] = (k.x0 + sb) + g.nx * ((k.y0 + yl) + g.ny * (k.z0 + zl));
                        g.nlpos[n] = (uint16_t)(t * 64 + sb);
                        g.nsize[n] = -1 - v;
                        g.npar[n] = n;
                    } else {
                        set_err(g, ERR_CAP);
                    }
                    s.par[id] = -1 - bidx;
                } else {
                    rw |= 1ull << sb;  // interior component: a finished cluster
                }
            }
            ++id;
        }
        g.root[(int64_t)b * R + t] = rw;
    }
    if (t == 0) g.bcount[b] = min(s.broff[R], g.cap);
    __syncthreads();

    uint16_t *F = g.face + (int64_t)b * g.fstride;
    const int lane = t & 63, wv = t >> 6;
    for (int r = wv; r < R; r += WG / 64) {
        const int yl = r & (g.BY - 1), zl = r >> g.lby;
        if (yl >= k.ey || zl >= k.ez) continue;
        const bool fyl = k.hyl && yl == 0, fyh = k.hyh && yl == k.ey - 1;
        const bool fzl = k.hzl && zl == 0, fzh = k.hzh && zl == k.ez - 1;
        if (!(fyl || fyh || fzl || fzh)) continue;
        const uint64_t w = s.occ[r];
        uint16_t e = NOSITE;
        if ((w >> lane) & 1ull) {
            const int run = s.rowoff[r] + __popcll(run_starts(w) & mask_le(lane)) - 1;
            const int bidx = -1 - s.par[root_of(s, run)];
            if (bidx >= 0 && bidx < g.cap)
                e = (uint16_t)bidx;
            else
                set_err(g, ERR_FACE);
        }
        if (fyl) F[f_ylo(g) + zl * 64 + lane] = e;
        if (fyh) F[f_yhi(g) + zl * 64 + lane] = e;
        if (fzl) F[f_zlo(g) + yl * 64 + lane] = e;
        if (fzh) F[f_zhi(g) + yl * 64 + lane] = e;
    }
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

// --------------------------------------------------------------------------
// phase: merge -- unite nodes across the brick's low x/y/z faces (the high
// faces are the low faces of the next bricks; wraps pair brick 0 with the
// last brick of a periodic axis)
// --------------------------------------------------------------------------

__device__ __forceinline__ void phase_merge(const Geo &g, int b) {
    const Brick k = brick_of(g, b);
    const int t = threadIdx.x;
    const int R = g.R;
    const uint16_t *F = g.face + (int64_t)b * g.fstride;
    if (k.hxl) {
        const int nbb = k.bx > 0 ? b - 1 : b + (g.nbx - 1);
        const uint16_t *G = g.face + (int64_t)nbb * g.fstride;
        for (int r = t; r < R; r += WG) {
            const int yl = r & (g.BY - 1), zl = r >> g.lby;
            if (yl >= k.ey || zl >= k.ez) continue;
            const uint16_t a = F[f_xlo(g) + r], c = G[f_xhi(g) + r];
            if (a == NOSITE || c == NOSITE) continue;
            if (yl > 0 && F[f_xlo(g) + r - 1] != NOSITE && G[f_xhi(g) + r - 1] != NOSITE) continue;
            g_unite(g, b * g.cap + a, nbb * g.cap + c);
        }
    }
    if (k.hyl) {
        const int nbb = k.by > 0 ? b - g.nbx : b + (g.nby - 1) * g.nbx;
        const uint16_t *G = g.face + (int64_t)nbb * g.fstride;
        for (int e = t; e < 64 * k.ez; e += WG) {
            const int x = e & 63;
            if (x >= k.ex) continue;
            const uint16_t a = F[f_ylo(g) + e], c = G[f_yhi(g) + e];
            if (a == NOSITE || c == NOSITE) continue;
            if (x > 0 && F[f_ylo(g) + e - 1] != NOSITE && G[f_yhi(g) + e - 1] != NOSITE) continue;
            g_unite(g, b * g.cap + a, nbb * g.cap + c);
        }
    }
    if (k.hzl) {
        const int nbb = k.bz > 0 ? b - g.nbx * g.nby : b + (g.nbz - 1) * g.nbx * g.nby;
        const uint16_t *G = g.face + (int64_t)nbb * g.fstride;
        for (int e = t; e < 64 * k.ey; e += WG) {
            const int x = e & 63;
            if (x >= k.ex) continue;
            const uint16_t a = F[f_zlo(g) + e], c = G[f_zhi(g) + e];
            if (a == NOSITE || c == NOSITE) continue;
            if (x > 0 && F[f_zlo(g) + e - 1] != NOSITE && G[f_zhi(g) + e - 1] != NOSITE) continue;
            g_unite(g, b * g.cap + a, nbb * g.cap + c);
        }
    }
}

// --------------------------------------------------------------------------
// phase: roots -- flatten every node of the brick to its root; roots mark
// their key site in the root bitmap, other nodes add their size to the root
// --------------------------------------------------------------------------

__device__ __forceinline__ void phase_roots(const Geo &g, int b) {
    const int cnt = g.bcount[b];
    for (int i = threadIdx.x; i < cnt; i += WG) {
        const int n = b * g.cap + i;
        const int r = g_root(g, n);
        if (r == n) {
            const int lp = g.nlpos[n];
            if ((lp >> 6) < g.R)
                atomicOr((unsigned long long *)(g.root + (int64_t)b * g.R + (lp >> 6)), 1ull << (lp & 63));
            else
                set_err(g, ERR_RANGE);
        } else {
            gl_st(g.npar + n, r);
            atomicAdd(g.nsize + r, g.nsize[n]);
        }
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
// phase: write -- redo the brick labelling, label = 1 + rank of the cluster's
// root site among all root sites in linear order; sizes from the root
// --------------------------------------------------------------------------

__device__ __forceinline__ void phase_write(const Geo &g, int b, LdsBrick &s) {
    const Brick k = brick_of(g, b);
    const int t = threadIdx.x;
    const int R = g.R;
    if (t < R) {
        const int64_t i = (int64_t)b * R + t;
        s.occ[t] = g.occ[i];
        s.rootw[t] = g.root[i];
        s.wpre[t] = g.wpre[i];
    }
    __syncthreads();
    brick_core(g, k, s);

    if (t < R) {
        const uint64_t w = s.occ[t];
        uint64_t m = run_starts(w);
        int id = s.rowoff[t];
        int bi = s.broff[t];
        while (m) {
            const int sb = __builtin_ctzll(m);
            m &= m - 1;
            const int v = s.par[id];
            if (v < 0) {
                int rank;
                int64_t size = -1;
                if (bflag_get(s, id)) {
                    const int bidx = bi++;
                    const int n = b * g.cap + min(bidx, g.cap - 1);
                    int rn = g.npar[n];
                    if ((unsigned)rn >= (unsigned)n_nodes(g)) {
                        set_err(g, ERR_RANGE);
                        rn = n;
                    }
                    if (rn == n) {
                        rank = s.wpre[t] + __popcll(s.rootw[t] & mask_lt(sb));
                        size = g.nsize[n];
                    } else {
                        const int bp = rn / g.cap;
                        const int lp = g.nlpos[rn];
                        const int64_t wi = (int64_t)bp * R + min(lp >> 6, R - 1);
                        rank = g.wpre[wi] + __popcll(g.root[wi] & mask_lt(lp & 63));
                    }
                } else {
                    rank = s.wpre[t] + __popcll(s.rootw[t] & mask_lt(sb));
                    size = -1 - v;
                }
                if (size >= 0 && g.sizes) {
                    if (rank >= 0 && (int64_t)rank < (n_sites(g) + 1) / 2)
                        g.sizes[rank] = size;
                    else
                        set_err(g, ERR_RANGE);
                }
                s.par[id] = -(rank + 1);
            }
            ++id;
        }
    }
    __syncthreads();

    const int lane = t & 63, wv = t >> 6;
    for (int r = wv; r < R; r += WG / 64) {
        const int yl = r & (g.BY - 1), zl = r >> g.lby;
        if (yl >= k.ey || zl >= k.ez) continue;
        const uint64_t w = s.occ[r];
        int lab = 0;
        if ((w >> lane) & 1ull) {
            const int run = s.rowoff[r] + __popcll(run_starts(w) & mask_le(lane)) - 1;
            lab = -s.par[root_of(s, run)];
        }
        if (lane < k.ex) g.labels[((int64_t)(k.z0 + zl) * g.ny + (k.y0 + yl)) * g.nx + k.x0 + lane] = lab;
    }
}

// --------------------------------------------------------------------------
// batched persistent loop: work items are (phase, job, item) triples laid
// out phase-major; a workgroup pops the next index, waits until every item
// of the previous phase of the same job has finished, runs the item, then
// publishes its completion.  An item only waits for items with smaller
// indices, popped earlier by workgroups that are already running, so the
// oldest unfinished item never waits and the queue always drains.  Every
// wait is bounded by a wall-clock limit that sets the sticky device error
// instead of hanging.
// --------------------------------------------------------------------------

constexpr int NPH = 8;  // pack, local, merge, roots, rowsum, scanblk, rowpre, write

struct BatchView {
    const Geo *jobs;
    const int32_t *itoff;   // [NPH][njobs + 1] item offsets of each job within a phase
    const int32_t *pstart;  // [NPH + 1] first item of each phase
    int32_t *done;          // [njobs][NPH] finished items
    int32_t *next;          // queue head
    int32_t *err;
    int32_t njobs;
    int32_t total;
    uint64_t wait_ticks;    // bound on one wait, in ticks of the 100 MHz clock
};

// Control flow of the loop is kept wave-uniform everywhere a barrier can
// follow: the queue and counter atomics are issued by the whole of wave 0
// with a non-zero operand in lane 0 only, and every value that steers a
// branch is broadcast with readfirstlane.  (A single-lane `if` around them
// let the compiler structure the loop exit as divergent, and waves then
// drifted apart across barriers.)
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ void persistent_loop(const BatchView &v, LdsBrick &s, int &s_item) {
    const int wave = uni(threadIdx.x >> 6);
    const int one = (threadIdx.x & 63) == 0 ? 1 : 0;
    for (;;) {
        if (wave == 0) s_item = uni(atomicAdd(v.next, one));
        __syncthreads();
        const int it = uni(s_item);
        __syncthreads();
        if (it >= v.total) break;
        int p = 0;
        while (p < NPH - 1 && it >= uni(v.pstart[p + 1])) ++p;
        const int rel = it - uni(v.pstart[p]);
        const int32_t *off = v.itoff + p * (v.njobs + 1);
        int lo = 0, hi = v.njobs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (uni(off[mid]) <= rel) lo = mid; else hi = mid;
        }
        const int j = lo;
        const int i = rel - uni(off[j]);
        const Geo &g = v.jobs[j];
        if (p > 0) {
            // every wave polls the counter as a scalar loop
            const int32_t *prev = v.itoff + (p - 1) * (v.njobs + 1);
            const int need = uni(prev[j + 1]) - uni(prev[j]);
            int32_t *cnt = v.done + j * NPH + (p - 1);
            const uint64_t t0 = wall_clock64();
            for (;;) {
                const int c = uni(__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
                if (c >= need) break;
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > v.wait_ticks) {
                    atomicOr(v.err, one ? ERR_LOOP : 0);
                    break;
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        switch (p) {
            case 0: phase_pack(g, i); break;
            case 1: phase_local(g, i, s); break;
            case 2: phase_merge(g, i); break;
            case 3: phase_roots(g, i); break;
            case 4: phase_rowsum(g, i, s.tmp); break;
            case 5: phase_scanblk(g, s.tmp); break;
            case 6: phase_rowpre(g, i, s.tmp); break;
            default: phase_write(g, i, s); break;
        }
        __threadfence();
        __syncthreads();
        if (wave == 0)
            __hip_atomic_fetch_add(v.done + j * NPH + p, one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace hk
