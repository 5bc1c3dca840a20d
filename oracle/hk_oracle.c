/*
 * Serial Hoshen-Kopelman oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct CPU reference that the GPU
 * path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Frijters, Krueger, Harting, "Parallelised Hoshen-Kopelman
 * algorithm for lattice-Boltzmann simulations", CPC 2014):
 *   - Sec. 2, occupancy condition: a site belongs to a cluster iff phi > 0;
 *     initial label 0 for the medium, -1 (here: "unvisited") for cluster sites.
 *   - Sec. 2, rules 1-3 applied in one raster pass, looking only backwards
 *     (no diagonal neighbours), equivalences kept in a label-of-labels table.
 *   - Sec. 3, equivalences stored as a singly linked list whose traversal ends
 *     at the lowest label; a new equivalence updates the list ending in the
 *     larger value.
 *   - Sec. 3, periodic boundaries: the wrap-around neighbours become extra
 *     equivalences (the serial analogue of the halo equivalences).
 *   - Sec. 2, final step: equivalences are compacted so that clusters use the
 *     labels 1..n, then applied in a last pass over the lattice.
 *   - Sec. 5: cluster sizes are the number of sites carrying each label.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes of the repository):
 *   - 3D raster order is x fastest, then y, then z; linear index
 *     i = x + nx*(y + ny*z).
 *   - Rule 3 takes the minimum over the *resolved* neighbour labels.
 *   - Wrap equivalences are added in a pass after the raster pass, for every
 *     axis whose periodic bit is set and whose length is at least 2.
 *   - Compaction numbers the surviving root labels in increasing order.  The
 *     root of each class is the label first created in it, i.e. the one
 *     created at the cluster's lowest linear site, so clusters come out
 *     numbered by their lowest linear site index.
 *   - The occupancy test is the IEEE single-precision comparison phi > 0
 *     (NaN and both zeros are empty, positive denormals are occupied).
 *
 * Parity status: pinned by the tests against brute-force flood fill,
 * a library routine (scipy.ndimage.label) with a separate wrap merge,
 * closed forms (empty, full, checkerboards, the paper's block checkerboard,
 * rows with gaps, serpentines, capsules) and invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HKO_OK 0
#define HKO_EINVAL -1
#define HKO_ETOOLARGE -2
#define HKO_ENOMEM -5

/* label-of-labels table: lol[l] == l marks the lowest label of a class */
typedef struct {
    int32_t *lol;
    int64_t cap;
    int32_t lmax;
} lol_table;

/* follow the list to its end, halving the path on the way (Sec. 3 allows
 * any traversal that ends at the lowest label of the class) */
static int32_t lol_find(lol_table *t, int32_t l)
{
    while (t->lol[l] != l) {
        t->lol[l] = t->lol[t->lol[l]];
        l = t->lol[l];
    }
    return l;
}

/* store the equivalence a == b: the list ending in the larger value is
 * redirected to the smaller one (Sec. 3) */
static void lol_union(lol_table *t, int32_t a, int32_t b)
{
    int32_t ra = lol_find(t, a);
    int32_t rb = lol_find(t, b);
    if (ra == rb)
        return;
    if (ra < rb)
        t->lol[rb] = ra;
    else
        t->lol[ra] = rb;
}

/* rule 1: a fresh label l_max + 1 */
static int lol_new(lol_table *t, int32_t *out)
{
    if ((int64_t)t->lmax + 1 >= t->cap) {
        int64_t ncap = t->cap * 2;
        int32_t *p = (int32_t *)realloc(t->lol, (size_t)ncap * sizeof(int32_t));
        if (!p)
            return HKO_ENOMEM;
        t->lol = p;
        t->cap = ncap;
    }
    t->lmax += 1;
    t->lol[t->lmax] = t->lmax;
    *out = t->lmax;
    return HKO_OK;
}

int64_t hk_oracle_max_clusters(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1)
        return 0;
    int64_t n = (int64_t)nx * ny * nz;
    return (n + 1) / 2;
}

/*
 * hk_oracle_label: label one lattice on the host.
 *   phi      [nz][ny][nx] float32, read only
 *   mask     bit 0: x periodic, bit 1: y periodic, bit 2: z periodic
 *   labels   [nz][ny][nx] int32 out: 0 for medium, 1..K for clusters
 *   n_clusters  out: K
 *   sizes    out, may be NULL: sizes[k-1] = number of sites labelled k;
 *            must hold hk_oracle_max_clusters() entries
 * Returns 0, or a negative code with nothing written on argument errors.
 */
int hk_oracle_label(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t mask,
                    int32_t *labels, int64_t *n_clusters, int64_t *sizes)
{
    if (!phi || !labels || !n_clusters)
        return HKO_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || mask > 7u)
        return HKO_EINVAL;
    const int64_t n = (int64_t)nx * ny * nz;
    if (n > INT32_MAX)
        return HKO_ETOOLARGE;

    lol_table t;
    t.cap = 1024;
    t.lol = (int32_t *)malloc((size_t)t.cap * sizeof(int32_t));
    if (!t.lol)
        return HKO_ENOMEM;
    t.lol[0] = 0;
    t.lmax = 0;

    const int64_t sy = nx, sz = (int64_t)nx * ny;

    /* initialisation (Sec. 2): 0 for the medium; cluster sites are handled
     * in the raster pass the moment they are visited */
    for (int64_t i = 0; i < n; ++i)
        labels[i] = 0;

    /* raster pass: rules 1-3 with backward neighbours -x, -y, -z, no wrap */
    for (int32_t z = 0; z < nz; ++z) {
        for (int32_t y = 0; y < ny; ++y) {
            for (int32_t x = 0; x < nx; ++x) {
                const int64_t i = x + sy * y + sz * z;
                if (!(phi[i] > 0.0f))
                    continue;
                int32_t nb[3];
                int cnt = 0;
                if (x > 0 && labels[i - 1] > 0)
                    nb[cnt++] = lol_find(&t, labels[i - 1]);
                if (y > 0 && labels[i - sy] > 0)
                    nb[cnt++] = lol_find(&t, labels[i - sy]);
                if (z > 0 && labels[i - sz] > 0)
                    nb[cnt++] = lol_find(&t, labels[i - sz]);
                if (cnt == 0) {
                    /* rule 1 */
                    int32_t l;
                    if (lol_new(&t, &l) != HKO_OK) {
                        free(t.lol);
                        return HKO_ENOMEM;
                    }
                    labels[i] = l;
                } else {
                    /* rules 2 and 3: smallest neighbour label, and record
                     * every pair of neighbour labels as equivalent */
                    int32_t m = nb[0];
                    for (int k = 1; k < cnt; ++k)
                        if (nb[k] < m)
                            m = nb[k];
                    labels[i] = m;
                    for (int k = 0; k < cnt; ++k)
                        if (nb[k] != m)
                            lol_union(&t, m, nb[k]);
                }
            }
        }
    }

    /* periodic boundaries: the site at coordinate n-1 and the site at 0 of
     * a wrapped axis are neighbours */
    if ((mask & 1u) && nx >= 2) {
        for (int32_t z = 0; z < nz; ++z)
            for (int32_t y = 0; y < ny; ++y) {
                const int64_t a = sy * y + sz * z, b = a + (nx - 1);
                if (labels[a] > 0 && labels[b] > 0)
                    lol_union(&t, labels[a], labels[b]);
            }
    }
    if ((mask & 2u) && ny >= 2) {
        for (int32_t z = 0; z < nz; ++z)
            for (int32_t x = 0; x < nx; ++x) {
                const int64_t a = x + sz * z, b = a + sy * (ny - 1);
                if (labels[a] > 0 && labels[b] > 0)
                    lol_union(&t, labels[a], labels[b]);
            }
    }
    if ((mask & 4u) && nz >= 2) {
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t x = 0; x < nx; ++x) {
                const int64_t a = x + sy * y, b = a + sz * (nz - 1);
                if (labels[a] > 0 && labels[b] > 0)
                    lol_union(&t, labels[a], labels[b]);
            }
    }

    /* compaction (Sec. 2): surviving class ends get 1..K in increasing
     * order, every other label takes the number of its class end */
    int32_t *canon = (int32_t *)malloc((size_t)(t.lmax + 1) * sizeof(int32_t));
    if (!canon) {
        free(t.lol);
        return HKO_ENOMEM;
    }
    int64_t k = 0;
    canon[0] = 0;
    for (int32_t l = 1; l <= t.lmax; ++l)
        if (lol_find(&t, l) == l)
            canon[l] = (int32_t)(++k);
    for (int32_t l = 1; l <= t.lmax; ++l)
        canon[l] = canon[lol_find(&t, l)];

    /* final pass: apply the equivalences, count sites per label (Sec. 5) */
    if (sizes)
        for (int64_t c = 0; c < k; ++c)
            sizes[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t l = canon[labels[i]];
        labels[i] = l;
        if (sizes && l > 0)
            sizes[l - 1] += 1;
    }
    *n_clusters = k;
    free(canon);
    free(t.lol);
    return HKO_OK;
}
