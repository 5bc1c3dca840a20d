/*
 * hk.h -- Hoshen-Kopelman cluster labelling of 3D lattices on MI355X (gfx950).
 *
 * The operation (Frijters, Krueger, Harting, "Parallelised Hoshen-Kopelman
 * algorithm for lattice-Boltzmann simulations", CPC 2014):
 *   - Sec. 2: a site x belongs to a cluster iff phi(x) > 0 (IEEE single
 *     precision: NaN and both zeros are medium, positive denormals and +inf
 *     are cluster sites); label 0 marks the medium.
 *   - Sec. 2: only face neighbours count (no diagonals), i.e. 6-connectivity.
 *   - Sec. 3: any axis may be periodic; the sites at coordinate n-1 and 0 of
 *     a periodic axis are then neighbours.
 *   - Sec. 2, final step with compaction: clusters are numbered 1..K; this
 *     library numbers them in order of their lowest linear site index
 *     i = x + nx*(y + ny*z) (x fastest), which is exactly the numbering the
 *     paper's serial raster pass produces after compaction.
 *   - Sec. 5: cluster sizes are the number of sites carrying each label.
 *   - Sec. 3: a lattice of V sites has at most V/2 (rounded up) clusters.
 *
 * Memory layout: phi and labels are C-contiguous [nz][ny][nx] arrays (a torch
 * tensor of shape (nz, ny, nx)).  periodic_mask bit 0 = x, bit 1 = y,
 * bit 2 = z.
 *
 * Ownership: every pointer below (phi, labels, n_clusters, sizes) is a DEVICE
 * pointer owned by the caller; the library never frees or reallocates it.
 * phi is read only and never used as scratch; labels must not alias phi.
 * The library owns a workspace per (device, stream), grown on demand; a
 * call that has to grow it synchronises that stream first (only then).
 *
 * Execution: all work is enqueued on `stream`; nothing is synchronised on
 * the host.  Outputs are valid once the stream has completed.
 *
 * Errors: arguments are validated synchronously; a failing call returns a
 * negative hk_status and enqueues/writes nothing.  Launch failures return
 * HK_ERR_HIP.  Device-side consistency checks (bounded loops, index guards)
 * never fault: they set a sticky flag readable with hk_device_error().  The
 * library never prints and never aborts.
 *
 * Thread safety: calls on different streams may run concurrently; calls on
 * one stream are serialised by the stream.
 */
#ifndef HK_H
#define HK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HK_OK = 0,
    HK_ERR_INVALID_ARG = -1,  /* null pointer, an edge < 1, mask > 7, n_jobs < 0 */
    HK_ERR_TOO_LARGE = -2,    /* nx*ny*nz > INT32_MAX, or no brick shape fits */
    HK_ERR_NO_WORKSPACE = -3, /* workspace too small while the stream is being captured */
    HK_ERR_HIP = -4,          /* a HIP runtime call or a launch failed */
    HK_ERR_DEVICE = -5        /* hk_device_error: a device-side check fired */
} hk_status;

/*
 * hk_label: label one lattice (Sec. 2 rules with the Sec. 3 periodic
 * equivalences and compaction).
 *   phi          [nz][ny][nx] float32, device, read only
 *   nx, ny, nz   edges, each >= 1, nx*ny*nz <= INT32_MAX
 *   periodic_mask  bits 0..2 = x, y, z periodic
 *   labels       [nz][ny][nx] int32, device, out: 0 or 1..K
 *   n_clusters   one int64, device, out: K
 *   sizes        int64, device, out: sizes[k-1] = #sites with label k for
 *                k = 1..K; must hold hk_max_clusters(nx, ny, nz) entries;
 *                entries >= K are left untouched.  May be NULL.
 */
int hk_label(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
             int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream);

/* One lattice of a batch; fields as in hk_label. */
typedef struct {
    const float *phi;
    int32_t nx, ny, nz;
    uint32_t periodic_mask;
    int32_t *labels;
    int64_t *n_clusters;
    int64_t *sizes;
} hk_job;

/*
 * hk_label_batched: label n_jobs independent lattices of any shapes with one
 * launch per phase on `stream`, each covering the bricks of every job (the
 * job table itself is a HOST array; it is copied to the device by the call,
 * from pinned memory, so a captured call is one copy node and nine kernel
 * nodes).  Each job's output is
 * identical to what hk_label gives for it alone.  Every job is validated
 * before anything is enqueued.  n_jobs == 0 is a no-op.
 */
int hk_label_batched(const hk_job *jobs, int32_t n_jobs, hipStream_t stream);

/* ceil(nx*ny*nz / 2): the Sec. 3 bound on the number of clusters, i.e. the
 * capacity `sizes` must have.  0 for invalid edges. */
int64_t hk_max_clusters(int32_t nx, int32_t ny, int32_t nz);

/* Device workspace bytes hk_label needs for this shape (< 0: invalid). */
int64_t hk_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);

/* Device workspace bytes hk_label_batched needs for these jobs. */
int64_t hk_batched_workspace_bytes(const hk_job *jobs, int32_t n_jobs);

/*
 * hk_reserve: make the workspace of `stream` (on the current device) at least
 * `bytes` large now, and set up the pinned staging arena that batched calls
 * use while a stream is being captured, so that later calls -- for instance
 * under hipGraph capture -- do not allocate.  Synchronises the stream if the
 * workspace must grow.  A call made during capture without enough reserved
 * workspace (or arena) returns HK_ERR_NO_WORKSPACE.  A captured graph refers
 * to the stream's workspace: it stays valid until the workspace grows or
 * hk_release is called, and it must not run concurrently with other calls
 * on the same stream's workspace.
 */
int hk_reserve(int64_t bytes, hipStream_t stream);

/* Free every workspace of every device (synchronises each device first). */
void hk_release(void);

/* Human-readable name of a status code (static string). */
const char *hk_status_string(int status);

/*
 * Brick shape used for the brick-local pass: 64 x by x bz sites (x extent
 * fixed to one 64-bit occupancy word per row).  by and bz must be powers of
 * two with by*bz in [1, 256].  hk_set_brick(0, 0) restores automatic choice
 * (autotuned table when one was loaded, else a size heuristic).
 */
int hk_set_brick(int32_t by, int32_t bz);
/* The brick the library would use for this shape (by, bz written out). */
int hk_get_brick(int32_t nx, int32_t ny, int32_t nz, int32_t *by, int32_t *bz);
/* Install one autotuned entry: lattices whose sizes fall in the same
 * power-of-two bucket as (nx, ny, nz) use brick (by, bz); (0, 0) removes
 * the entry of that bucket. */
int hk_set_brick_for_shape(int32_t nx, int32_t ny, int32_t nz, int32_t by, int32_t bz);

/*
 * Per-kernel timing (a tracing aid, off by default).  While enabled, every
 * hk_label call records a HIP event on its own stream before each of its
 * kernels and after the last one.  hk_profile_read synchronises on those
 * events, writes into ms[i] the milliseconds spent in phase i summed over
 * all calls made since the previous read (n = capacity of ms), the number
 * of such calls into *calls, and forgets them.  hk_phase_count() phases
 * exist; hk_phase_name(i) names the kernel of phase i.
 */
int hk_profile_enable(int32_t enable);
int hk_profile_read(float *ms, int32_t n, int32_t *calls);
int32_t hk_phase_count(void);
const char *hk_phase_name(int32_t i);

/*
 * hk_device_error: synchronise `stream`, then report and clear the sticky
 * device-side check flag of its workspace (0 = none fired).  Returns HK_OK,
 * or HK_ERR_DEVICE when a flag was set (code written to *code if non-NULL).
 */
int hk_device_error(hipStream_t stream, int32_t *code);

#ifdef __cplusplus
}
#endif

#endif /* HK_H */
