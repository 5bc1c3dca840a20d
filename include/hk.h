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
    HK_ERR_DEVICE = -5,       /* hk_device_error: a device-side check fired */
    HK_ERR_TIMEOUT = -6       /* hk_server_wait / hk_server_drain: time limit reached */
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
 * The call enqueues kernels only (no copies, no memsets), so it may be
 * captured into a hipGraph once the stream's workspace is large enough
 * (an earlier call of the same shape on the stream, or hk_reserve).
 */
int hk_label(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
             int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream);

/* Occupancy predicates of hk_label_pred. */
typedef enum {
    HK_PRED_GT = 0, /* float32 field: occupied iff field > param */
    HK_PRED_EQ = 1, /* float32 field: occupied iff field == param */
    HK_PRED_U8 = 2  /* uint8 field: occupied iff field != 0 (param unused) */
} hk_predicate;

/*
 * hk_label_pred: hk_label with another occupancy condition.  Sec. 2 labels
 * the sites where phi > 0; the interior detection of Sec. 6 labels the sites
 * whose proximity value still equals the far-field value (HK_PRED_EQ with
 * that value), and a caller may hold a threshold other than 0 or a ready
 * byte mask.  Comparisons follow IEEE single precision and are decided on
 * the bits (no flush-to-zero mode changes them): NaN sites are never
 * occupied, +0 equals -0, denormals compare by value.
 *   field        [nz][ny][nx] float32 (HK_PRED_GT, HK_PRED_EQ) or uint8
 *                (HK_PRED_U8), device, read only
 *   predicate    an hk_predicate value
 *   param        the threshold or value; NaN is rejected for GT and EQ.
 *                HK_PRED_GT with param +-0 is exactly hk_label.
 * Other arguments, outputs, workspace and errors as in hk_label.
 */
int hk_label_pred(const void *field, int32_t predicate, float param, int32_t nx, int32_t ny, int32_t nz,
                  uint32_t periodic_mask, int32_t *labels, int64_t *n_clusters, int64_t *sizes, hipStream_t stream);

/*
 * Incremental relabelling of a field that changes little from one call to
 * the next (a lattice-Boltzmann field between time steps, Sec. 5 and 6: the
 * labelling runs every step on a slowly moving interface).  A state object
 * owns a workspace for one lattice shape and keeps, between calls, each
 * brick's local labelling; a call labels anew only the bricks whose
 * occupancy changed since the previous call on the same state, restores the
 * others, and runs the global phases over all.  Every call's outputs are
 * identical to what hk_label gives for the same field.
 *
 * hk_incr_create: a state for [nz][ny][nx] lattices with the given periodic
 *   mask, on the current device; *out receives it (NULL on error).  The
 *   workspace is allocated here (hipMalloc), about the size of hk_label's
 *   plus 4 B per node slot and 8 B per brick row.  Errors as for hk_label,
 *   HK_ERR_HIP when the allocation fails.
 * hk_incr_label: label `phi` ([nz][ny][nx] float32, device) into labels,
 *   n_clusters and sizes as hk_label does.  relabelled: one int64, device,
 *   out, or NULL: the number of bricks labelled anew by this call (all of
 *   them on the first call).  Calls on one state must be on its device and
 *   must not overlap (one stream, or ordered by the caller); the first call
 *   labels every brick.  Nothing is allocated.
 * hk_incr_device_error: as hk_device_error, for the state's own check flag.
 * hk_incr_destroy: synchronise the state's device and free the state.
 */
typedef struct hk_incr hk_incr;
int hk_incr_create(int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, hk_incr **out);
int hk_incr_label(hk_incr *state, const float *phi, int32_t *labels, int64_t *n_clusters, int64_t *sizes,
                  int64_t *relabelled, hipStream_t stream);
int hk_incr_device_error(hk_incr *state, hipStream_t stream, int32_t *code);
void hk_incr_destroy(hk_incr *state);

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
 * from pinned memory, so a captured call is one copy node and eight kernel
 * nodes).  Each job's output is
 * identical to what hk_label gives for it alone.  Every job is validated
 * before anything is enqueued.  n_jobs == 0 is a no-op.
 */
int hk_label_batched(const hk_job *jobs, int32_t n_jobs, hipStream_t stream);

/*
 * hk_classify: Sec. 6, last step of the detection of capsule interiors --
 * the HK pass has labelled the sites that kept the far-field proximity
 * value (labels, from hk_label on the same lattice: 0 = membrane site,
 * 1..K = cluster); each cluster is now judged by the proximity values of
 * the membrane sites around it.
 *   I            [nz][ny][nx] float32, device, read only: proximity value,
 *                negative on the interior side of a membrane, positive on
 *                the exterior side (read only at sites with label 0)
 *   labels       [nz][ny][nx] int32, device, read only
 *   n_clusters   one int64, device: K (as hk_label wrote it; read on the
 *                device, so no host synchronisation is needed in between)
 *   neg, pos     int64, device, out: for k = 1..K, the number of border
 *                pairs of cluster k -- face-adjacent (cluster site, label-0
 *                site) pairs, wrapping on the periodic axes, one pair on a
 *                periodic axis of length 2 -- whose I is < 0 / > 0; the
 *                sign is taken on the bits (denormals count, +-0 and NaN
 *                count for neither side)
 *   inside       int8, device, out: 1 if neg > pos (interior), 0 if
 *                pos > neg (exterior), -1 on a tie (or no border at all)
 * neg, pos and inside must hold hk_max_clusters(nx, ny, nz) entries;
 * entries >= K are left untouched.  Errors as for hk_label.
 */
int hk_classify(const float *I, const int32_t *labels, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
                const int64_t *n_clusters, int64_t *neg, int64_t *pos, int8_t *inside, hipStream_t stream);

/*
 * hk_droplet_stats: Sec. 5 -- cluster sizes as the radius of the sphere of
 * the same volume, R = (3 s / (4 pi))^(1/3) lattice units, over the clusters
 * of at least min_size sites.
 *   sizes         int64 [max_clusters], device, read only (hk_label output)
 *   n_clusters    one int64, device: K (entries >= min(K, max_clusters) are
 *                 not read)
 *   r_max, n_bins histogram over [0, r_max) in n_bins (1..2048) bins of
 *                 width w = r_max / n_bins; the last bin also takes R >= r_max
 *   hist          int64 [n_bins], device, out: clusters per bin.  The bin is
 *                 decided on the size: s >= (4 pi / 3) e^3 <=> R >= e, with
 *                 the edge thresholds computed in IEEE double as
 *                 c * (e * e * e), c = 4.0 * pi / 3.0, e = i * w -- exact.
 *   counts        int64 [2], device, out: number of clusters counted, sum of
 *                 their sizes
 *   sums          double [3], device, out: sums of R, R^2, R^3 (summation
 *                 order unspecified: these carry rounding)
 * No host synchronisation; errors as for hk_label.
 */
int hk_droplet_stats(const int64_t *sizes, const int64_t *n_clusters, int64_t max_clusters, int64_t min_size,
                     double r_max, int32_t n_bins, int64_t *hist, int64_t *counts, double *sums,
                     hipStream_t stream);

/*
 * hk_label_droplets: Sec. 2 labelling (as hk_label) with the Sec. 5
 * droplet statistics gathered in the same pass that finalises the cluster
 * sizes (no second pass over `sizes`, which may here be NULL).
 *   phi .. sizes  as for hk_label
 *   min_size, r_max, n_bins, hist, counts, sums
 *                 as for hk_droplet_stats, over all K clusters: the same
 *                 bin counts and counts exactly, the sums of R^k up to the
 *                 order of summation
 * hist, counts and sums are written (not accumulated).  Uses the stream's
 * workspace as hk_label, plus 8 * 256 * (n_bins + 5) bytes.  No host
 * synchronisation; errors as for hk_label and hk_droplet_stats.
 */
int hk_label_droplets(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
                      int32_t *labels, int64_t *n_clusters, int64_t *sizes, int64_t min_size, double r_max,
                      int32_t n_bins, int64_t *hist, int64_t *counts, double *sums, hipStream_t stream);

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
 * Brick autotuner.  hk_autotune runs hk_label on this lattice once per
 * candidate brick shape (powers of two, by*bz between min(64, what the
 * lattice allows) and 256) -- one untimed call, then `reps` timed calls
 * between HIP events on `stream`, which it synchronises -- and installs the
 * fastest shape for the lattice's size bucket (as hk_set_brick_for_shape).
 * It writes the shape to *by, *bz and its mean time in ms to *ms (each may
 * be NULL).  The outputs end holding the result of one more call with the
 * chosen shape, identical to hk_label's.  hk_autotune_batched does the same
 * with hk_label_batched over `jobs`, choosing one shape for the whole batch
 * and installing it for the bucket of every job.  While a tuning run lasts
 * it overrides the brick choice of every other call.
 */
int hk_autotune(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, int32_t *labels,
                int64_t *n_clusters, int64_t *sizes, int32_t reps, hipStream_t stream, int32_t *by, int32_t *bz,
                float *ms);
int hk_autotune_batched(const hk_job *jobs, int32_t n_jobs, int32_t reps, hipStream_t stream, int32_t *by,
                        int32_t *bz, float *ms);
/* Write the tuned table to a text file ("log2(nx) log2(ny) log2(nz) by bz"
 * per line) / install the entries of such a file (a malformed file installs
 * nothing and returns HK_ERR_INVALID_ARG). */
int hk_tune_save(const char *path);
int hk_tune_load(const char *path);

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

/*
 * hk_debug_counters: synchronise `stream`, then write into counts[0..n) and
 * clear the fallback counters of its workspace, summed over the hk_label,
 * hk_label_pred and hk_label_batched calls on that stream since the last
 * read.  Each counts the times a bounded fast structure was full and a
 * slower exact path took over; results never depend on them:
 *   [0] face pairs united where found (a brick's LDS pair list was full)
 *   [1] node sizes added to their root directly (the LDS hash of a group of
 *       bricks ran out of probes)
 *   [2] bricks whose list of equivalences overflowed (their overlaps are
 *       united again directly)
 *   [3] bricks whose run slots did not fit the write phase's LDS (read from
 *       global memory instead)
 * Entries at index >= 4 are written as 0.
 */
int hk_debug_counters(hipStream_t stream, int64_t *counts, int32_t n);

/*
 * ------------------------------------------------------------------------
 * Labelling server (continuous batching on one device).
 *
 * A server owns one device arena of `arena_bytes`, allocated at creation;
 * nothing is allocated per request.  Each request (a device-resident phi,
 * Sec. 2 condition, Sec. 3 periodicity as in hk_label) takes
 * hk_server_footprint() arena bytes: its outputs, labels [N] int32 and sizes
 * [ceil(N/2)] int64 (the Sec. 3 bound), which stay in the arena until
 * hk_server_release, plus its share of the workspace of the batch it runs
 * in, freed when that batch completes.  Requests are admitted first come
 * first served when arena space and one of `n_slots` batch slots are free;
 * a free slot takes the longest prefix of the waiting queue that fits (at
 * most max_batch_jobs requests) and labels it with the batched kernels on
 * its own stream, so up to n_slots batches run concurrently and requests
 * that arrive while others run join the next batch.  A scheduler thread,
 * started by hk_server_create and joined by hk_server_destroy, does the
 * admission and polls completion.
 *
 * Ownership: phi is the caller's and must stay valid and unchanged until
 * the request is done (hk_server_poll returns 1) or failed.  hk_server_submit
 * takes phi as complete; when phi may still be in the making on a stream,
 * submit it with hk_server_submit_after and that stream (the legacy null
 * stream included): when that stream has work pending at submission, the
 * server records an event on it and the batch that reads phi waits for that
 * event on the device (an idle stream needs no wait).  Output
 * pointers from hk_server_result point into the arena and are valid until
 * hk_server_release of that ticket.  Results are identical to hk_label of
 * the same lattice alone.
 *
 * Latency of a request = time the scheduler observed its batch complete -
 * arrival, where arrival is the `arrival_ns` given to hk_server_submit on
 * the hk_server_now_ns() clock (0 = the submission time).  A request is not
 * admitted before its arrival time, so an arrival trace can be replayed by
 * submitting it ahead of time (in arrival order: admission is in submission
 * order).
 *
 * Errors: invalid arguments return HK_ERR_INVALID_ARG, a request larger
 * than the whole arena HK_ERR_TOO_LARGE (at submission).  Every request of
 * a batch has its own device-side check word: a check that fires fails that
 * request alone (HK_ERR_DEVICE) and the others of its batch complete.  A
 * failure of the batch itself (a launch or copy that fails, or an
 * asynchronous error its completion event reports) fails every request of
 * that batch with HK_ERR_HIP and no other.  poll/wait/result return a failed
 * request's status, wait also when the failure falls on its deadline.
 * All calls are thread-safe.
 * ------------------------------------------------------------------------
 */
typedef struct hk_server hk_server;

typedef struct {
    int64_t submitted, completed, failed;  /* since creation or the last reset */
    int64_t batches;
    double mean_batch_jobs;
    int64_t pending, running;              /* now */
    int64_t sites_completed;
    int64_t arena_bytes, arena_in_use, arena_peak;
    int64_t latency_samples;               /* completed requests */
    int64_t latency_p50_ns, latency_p99_ns, latency_max_ns;  /* nearest rank */
    double latency_mean_ns;
    int64_t span_ns;                       /* first batch launch to last completion */
} hk_server_stats;

/* n_slots in [1, 16] batches in flight; max_batch_jobs in [1, 65536]. */
int hk_server_create(int64_t arena_bytes, int32_t n_slots, int32_t max_batch_jobs, hk_server **out);
/* The same scheduler with a simulated device (no HIP call is made): a batch
 * completes batch_fixed_ns + ns_per_site * (its sites) after its launch and
 * every K is 0; output pointers are arena offsets.  phi may be NULL.  For
 * exercising admission and batching without a GPU. */
int hk_server_create_simulated(int64_t arena_bytes, int32_t n_slots, int32_t max_batch_jobs, int64_t batch_fixed_ns,
                               double ns_per_site, hk_server **out);
/* Arena bytes one request of this shape needs when it runs alone. */
int64_t hk_server_footprint(int32_t nx, int32_t ny, int32_t nz);
/* The server clock (steady, nanoseconds). */
int64_t hk_server_now_ns(void);
int hk_server_submit(hk_server *s, const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
                     int64_t arrival_ns, uint64_t *ticket);
int hk_server_submit_after(hk_server *s, const float *phi, int32_t nx, int32_t ny, int32_t nz,
                           uint32_t periodic_mask, int64_t arrival_ns, hipStream_t producer, uint64_t *ticket);
/* Simulated servers only: plant a failure on a waiting request, for tests
 * of the failure paths.  HK_ERR_DEVICE fires that request's own device
 * check; any other negative status is reported by the completion of the
 * whole batch it runs in.  HK_ERR_INVALID_ARG on a real server. */
int hk_server_sim_fail(hk_server *s, uint64_t ticket, int32_t status);
/* 1 done, 0 waiting or running, < 0 failed (its status) or unknown ticket. */
int hk_server_poll(hk_server *s, uint64_t ticket);
/* Block until the request is done (HK_OK), failed (its status) or timeout_ns passed (HK_ERR_TIMEOUT). */
int hk_server_wait(hk_server *s, uint64_t ticket, int64_t timeout_ns);
/* Block until no request waits or runs. */
int hk_server_drain(hk_server *s, int64_t timeout_ns);
/* Device pointers of a done request's outputs, its K and latency (any out pointer may be NULL). */
int hk_server_result(hk_server *s, uint64_t ticket, int32_t **labels, int64_t *n_clusters, int64_t **sizes,
                     int64_t *latency_ns);
/* Free a done or failed request's outputs, or withdraw a waiting one; a running one is refused. */
int hk_server_release(hk_server *s, uint64_t ticket);
int hk_server_read_stats(hk_server *s, hk_server_stats *out);
int hk_server_reset_stats(hk_server *s);
/* Stop the scheduler, wait for running batches, free the arena; waiting requests are dropped. */
int hk_server_destroy(hk_server *s);

/*
 * hk_label_noalloc: hk_label for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, hosts that forbid
 * allocation).  Same arguments, outputs and argument checks as hk_label,
 * computed by the same kernels, but the workspace is carved from a fixed
 * 64 MiB device array inside the library (one per device, held until the
 * process ends) and no call allocates or frees anything.  Lattices whose
 * workspace does not fit it (a few million sites, depending on the shape)
 * return HK_ERR_TOO_LARGE with no writes.  All calls on one device share
 * the array: calls that overlap on one device race and must be serialised
 * by the caller.  A device-side check that fires leaves *n_clusters equal to
 * minus its code (hk_device_error does not see this array).
 */
int hk_label_noalloc(const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask, int32_t *labels,
                     int64_t *n_clusters, int64_t *sizes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HK_H */
