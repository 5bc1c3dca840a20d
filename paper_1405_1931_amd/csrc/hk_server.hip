// Labelling server: continuous batching of labelling requests on one device.
//
// Requests carry a device-resident phi.  The server owns one device arena,
// allocated once at creation, from which it carves each request's outputs
// (labels, sizes) and each launched batch's workspace; admission is by that
// footprint, first come first served.  Up to `n_slots` batches are in flight
// at once, each on its own stream, so their kernels overlap on the device.
// A scheduler thread polls the in-flight batches; whenever one completes it
// frees the batch workspace and immediately launches the longest prefix of
// the waiting queue that fits the free slots and arena space -- requests
// that arrived while others were on the GPU join the next batch as soon as
// a slot and memory are free.  Outputs stay in the arena until the caller
// releases the request.
//
// Latency of a request = completion observed by the scheduler - arrival
// (the arrival time the caller passes, or the submission time).  A request
// whose arrival time lies ahead is held until then, so a recorded arrival
// trace can be replayed by submitting it ahead of time.
//
// A simulated executor (no HIP call at all) stands in for the device so that
// the admission, batching and accounting logic can be exercised anywhere:
// a batch then "runs" for fixed_ns + ns_per_site * sites of wall time, and
// a failure can be planted on a request (its own device check, or an error
// of its whole batch) to exercise the failure paths.
//
// Failure isolation: every job of a batch has its own device-check word, so
// a check that fires fails that job alone; an error of the batch itself (a
// launch or copy that fails, or an asynchronous error reported by its
// completion event) fails every job of that batch and no other.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hk.h"
#include "hk_device.h"

namespace hk {

int plan_lattice_ext(int32_t nx, int32_t ny, int32_t nz, uint32_t mask, Geo *g);
int64_t lattice_bytes(const Geo &g);
std::mutex &workspace_mutex();
int plan_batched(const hk_job *jobs, int n_jobs, std::vector<Geo> *geos, int64_t *bytes);
int enqueue_batched(const hk_job *jobs, int n_jobs, const std::vector<Geo> &geos, char *ws, int32_t *err,
                    int64_t err_stride, uint32_t *dbg, hipStream_t stream);

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t al(int64_t v) { return (v + 255) / 256 * 256; }

// first-fit allocator over [0, size) with coalescing; offsets only
class Arena {
public:
    explicit Arena(int64_t size) : size_(size) {
        if (size > 0) free_[0] = size;
    }
    // returns the offset, or -1 when no free block is large enough
    int64_t alloc(int64_t bytes) {
        bytes = al(std::max<int64_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = al(std::max<int64_t>(bytes, 1));
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    int64_t size() const { return size_; }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

private:
    int64_t size_, used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;
};

enum class State { Pending, Running, Done, Failed };

struct Request {
    const float *phi = nullptr;
    int32_t nx = 0, ny = 0, nz = 0;
    uint32_t mask = 0;
    int64_t sites = 0;
    int64_t ws_bytes = 0;   // this lattice's share of a batch workspace
    int64_t lab_bytes = 0;  // labels, then sizes, in one output block
    int64_t out_bytes = 0;
    int64_t out_off = -1;
    int64_t arrival = 0, done = 0;
    int64_t k = -1;
    int status = HK_OK;
    State state = State::Pending;
    hipEvent_t ready = nullptr;  // recorded on the producer stream at submission, or null
    hipStream_t producer = nullptr;  // the stream `ready` was recorded on
    int sim_fail = HK_OK;        // simulated servers: the failure planted on this request
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int64_t *host = nullptr;  // pinned: K of every job, then every job's device check word
    bool busy = false;
    int64_t off = -1, bytes = 0;
    int64_t sim_done = 0;
    int sim_error = HK_OK;  // simulated: the error the batch's completion reports
    std::vector<uint64_t> tickets;
};

// bytes of a batch block for n jobs whose lattice shares sum to ws: the
// workspace (job table included), then K of every job, then every job's
// check word (8 bytes each)
int64_t batch_tail_bytes(int n) { return al((int64_t)2 * n * 8); }
int64_t batch_block_bytes(int n, int64_t ws_shares) {
    const int64_t table = al((int64_t)n * (int64_t)sizeof(Geo)) + al((int64_t)NPH * (n + 1) * 4);
    return al(ws_shares + table) + batch_tail_bytes(n);
}

}  // namespace
}  // namespace hk

using namespace hk;

struct hk_server {
    bool sim = false;
    int64_t sim_fixed_ns = 0;
    double sim_ns_per_site = 0.0;
    int dev = 0;
    char *base = nullptr;  // device arena (null when simulated)
    Arena arena{0};
    int max_batch = 1;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable work_cv, done_cv;
    bool stop = false;
    std::thread thread;

    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> queue;

    // statistics since the last reset
    std::vector<int64_t> lat;
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0, batched_jobs = 0, sites_done = 0;
    int64_t first_launch = 0, last_done = 0;

    std::vector<hipEvent_t> event_pool;  // request events, reused

    // ---------------------------------------------------------------- batches
    // 1: the batch completed; 0: still running; < 0: the batch failed with
    // that status (any completion-event result but "not ready" is an error)
    int slot_state(Slot &s) {
        if (sim) return now_ns() >= s.sim_done ? (s.sim_error != HK_OK ? s.sim_error : 1) : 0;
        const hipError_t e = hipEventQuery(s.ev);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        (void)hipGetLastError();
        return HK_ERR_HIP;
    }

    void finish(Slot &s) {
        const int64_t t = now_ns();
        const int n = (int)s.tickets.size();
        for (int j = 0; j < n; ++j) {
            Request &r = reqs[s.tickets[j]];
            r.done = t;
            // this job's own device check word
            const int64_t check = sim ? (r.sim_fail == HK_ERR_DEVICE ? 1 : 0) : s.host[n + j];
            if (check != 0) {
                r.state = State::Failed;
                r.status = HK_ERR_DEVICE;
                ++failed;
            } else {
                r.state = State::Done;
                r.k = sim ? 0 : s.host[j];
                ++completed;
                sites_done += r.sites;
                lat.push_back(t - r.arrival);
            }
        }
        last_done = t;
        arena.release(s.off, s.bytes);
        s.busy = false;
        s.tickets.clear();
    }

    void fail_batch(Slot &s, int status) {
        for (uint64_t tk : s.tickets) {
            Request &r = reqs[tk];
            r.state = State::Failed;
            r.status = status;
            r.done = now_ns();
            ++failed;
        }
        arena.release(s.off, s.bytes);
        s.busy = false;
        s.tickets.clear();
    }

    hipEvent_t take_event() {
        hipEvent_t e = nullptr;
        if (!event_pool.empty()) {
            e = event_pool.back();
            event_pool.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
        }
        return e;
    }

    // launch the longest prefix of the queue that fits this slot and the arena.
    // Called with `lk` held; the batch is taken under it, then the lock is
    // released while the batch is planned and enqueued (host work of some
    // tens of microseconds that submissions need not wait for: only this
    // thread touches the slot and the taken requests until they finish), and
    // taken again for the bookkeeping.
    bool launch(Slot &s, std::unique_lock<std::mutex> &lk) {
        std::vector<uint64_t> take;
        int64_t shares = 0;
        const int64_t now = now_ns();
        for (uint64_t tk : queue) {
            if ((int)take.size() >= max_batch) break;
            Request &r = reqs[tk];
            if (r.arrival > now) break;  // not arrived yet: it and everything behind it wait
            const int64_t off = arena.alloc(r.out_bytes);
            if (off < 0) break;
            r.out_off = off;
            take.push_back(tk);
            shares += r.ws_bytes;
        }
        // the batch block; shed jobs from the tail until it fits
        int64_t boff = -1, bbytes = 0;
        while (!take.empty()) {
            bbytes = batch_block_bytes((int)take.size(), shares);
            boff = arena.alloc(bbytes);
            if (boff >= 0) break;
            Request &r = reqs[take.back()];
            arena.release(r.out_off, r.out_bytes);
            r.out_off = -1;
            shares -= r.ws_bytes;
            take.pop_back();
        }
        if (take.empty()) return false;
        queue.erase(queue.begin(), queue.begin() + (int64_t)take.size());
        s.busy = true;
        s.off = boff;
        s.bytes = bbytes;
        s.tickets = take;
        const int n = (int)take.size();
        for (uint64_t tk : take) reqs[tk].state = State::Running;
        ++batches;
        batched_jobs += n;
        const int64_t t = now_ns();
        if (!first_launch) first_launch = t;
        if (sim) {
            int64_t sites = 0;
            s.sim_error = HK_OK;
            for (uint64_t tk : take) {
                sites += reqs[tk].sites;
                if (reqs[tk].sim_fail != HK_OK && reqs[tk].sim_fail != HK_ERR_DEVICE) s.sim_error = reqs[tk].sim_fail;
            }
            s.sim_done = t + sim_fixed_ns + (int64_t)(sim_ns_per_site * (double)sites);
            return true;
        }
        // real device: job descriptors into the arena
        char *block = base + boff;
        const int64_t ws_bytes = bbytes - batch_tail_bytes(n);
        int64_t *kbuf = (int64_t *)(block + ws_bytes);
        std::vector<hk_job> jobs(n);
        for (int j = 0; j < n; ++j) {
            Request &r = reqs[take[j]];
            char *out = base + r.out_off;
            jobs[j] = hk_job{r.phi, r.nx, r.ny, r.nz, r.mask, (int32_t *)out, kbuf + j, (int64_t *)(out + r.lab_bytes)};
        }
        // the batch reads each phi only after the work its producer stream had
        // enqueued when the request was submitted.  Of the requests from one
        // producer stream the latest event covers the earlier ones (stream
        // order), so the batch waits once per producer stream.
        std::vector<hipEvent_t> waits, used;
        {
            std::vector<hipStream_t> seen;
            for (auto it = take.rbegin(); it != take.rend(); ++it) {
                Request &r = reqs[*it];
                if (!r.ready) continue;
                if (std::find(seen.begin(), seen.end(), r.producer) == seen.end()) {
                    seen.push_back(r.producer);
                    waits.push_back(r.ready);
                }
                used.push_back(r.ready);
                r.ready = nullptr;
            }
        }
        lk.unlock();
        std::vector<Geo> geos;
        int64_t need = 0;
        int rc = plan_batched(jobs.data(), n, &geos, &need);
        if (rc == HK_OK && need > ws_bytes) rc = HK_ERR_NO_WORKSPACE;
        for (hipEvent_t e : waits)
            if (rc == HK_OK && hipStreamWaitEvent(s.stream, e, 0) != hipSuccess) rc = HK_ERR_HIP;
        if (rc == HK_OK && hipMemsetAsync(kbuf + n, 0, (size_t)n * 8, s.stream) != hipSuccess) rc = HK_ERR_HIP;
        if (rc == HK_OK) {
            std::lock_guard<std::mutex> wl(workspace_mutex());
            rc = enqueue_batched(jobs.data(), n, geos, block, (int32_t *)(kbuf + n), 8, nullptr, s.stream);
        }
        if (rc == HK_OK &&
            hipMemcpyAsync(s.host, kbuf, (size_t)(2 * n) * 8, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            rc = HK_ERR_HIP;
        if (rc == HK_OK && hipEventRecord(s.ev, s.stream) != hipSuccess) rc = HK_ERR_HIP;
        if (rc != HK_OK) (void)hipStreamSynchronize(s.stream);
        lk.lock();
        // the events may be recorded again once the stream-ordered waits are enqueued
        for (hipEvent_t e : used) event_pool.push_back(e);
        if (rc != HK_OK) {
            // nothing observable was launched for these jobs: report and free
            for (uint64_t tk : take) {
                Request &r = reqs[tk];
                arena.release(r.out_off, r.out_bytes);
                r.out_off = -1;
            }
            fail_batch(s, rc);
        }
        return true;
    }

    void run() {
        if (!sim) (void)hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            bool progress = false;
            for (Slot &s : slots) {
                if (!s.busy) continue;
                const int st = slot_state(s);
                if (st == 1) {
                    finish(s);
                    progress = true;
                } else if (st < 0) {
                    // the batch itself failed: its jobs, and only they, fail
                    for (uint64_t tk : s.tickets) {
                        Request &r = reqs[tk];
                        arena.release(r.out_off, r.out_bytes);
                        r.out_off = -1;
                    }
                    fail_batch(s, st);
                    progress = true;
                }
            }
            if (progress) done_cv.notify_all();
            for (Slot &s : slots) {
                if (queue.empty()) break;
                if (!s.busy && launch(s, lk)) progress = true;
            }
            if (progress) {
                done_cv.notify_all();
                continue;
            }
            bool inflight = false;
            for (Slot &s : slots) inflight |= s.busy;
            // the queue head may be a request whose arrival time is still ahead
            const int64_t head = queue.empty() ? 0 : reqs[queue.front()].arrival;
            if (inflight)
                work_cv.wait_for(lk, std::chrono::microseconds(20));
            else if (head > now_ns())
                work_cv.wait_for(lk, std::chrono::nanoseconds(std::min<int64_t>(head - now_ns(), 20000)));
            else if (queue.empty())
                work_cv.wait(lk);
            else
                work_cv.wait_for(lk, std::chrono::microseconds(20));  // head waits for arena space
        }
    }

    void reset_stats() {
        lat.clear();
        submitted = completed = failed = batches = batched_jobs = sites_done = 0;
        first_launch = last_done = 0;
        arena.reset_peak();
    }
};

namespace {

// arena bytes of one request's outputs: labels [N] int32 then sizes [ceil(N/2)] int64
void output_bytes(int64_t n, int64_t *lab, int64_t *total) {
    *lab = al(4 * n);
    *total = *lab + al(8 * std::max<int64_t>(1, (n + 1) / 2));
}

int create(int64_t arena_bytes, int32_t n_slots, int32_t max_batch, bool sim, int64_t fixed_ns, double ns_site,
           hk_server **out) {
    if (!out || arena_bytes <= 0 || n_slots < 1 || n_slots > 16 || max_batch < 1 || max_batch > 65536 ||
        fixed_ns < 0 || ns_site < 0)
        return HK_ERR_INVALID_ARG;
    *out = nullptr;
    hk_server *s = new hk_server();
    s->sim = sim;
    s->sim_fixed_ns = fixed_ns;
    s->sim_ns_per_site = ns_site;
    s->max_batch = max_batch;
    s->arena = Arena(al(arena_bytes));
    s->slots.resize(n_slots);
    if (!sim) {
        bool ok = hipGetDevice(&s->dev) == hipSuccess;
        void *p = nullptr;
        ok = ok && hipMalloc(&p, (size_t)al(arena_bytes)) == hipSuccess;
        s->base = (char *)p;
        for (Slot &sl : s->slots) {
            if (!ok) break;
            void *h = nullptr;
            ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess &&
                 hipHostMalloc(&h, (size_t)(2 * max_batch) * 8, hipHostMallocDefault) == hipSuccess;
            sl.host = (int64_t *)h;
        }
        if (!ok) {
            for (Slot &sl : s->slots) {
                if (sl.host) (void)hipHostFree(sl.host);
                if (sl.ev) (void)hipEventDestroy(sl.ev);
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
            }
            if (s->base) (void)hipFree(s->base);
            (void)hipGetLastError();
            delete s;
            return HK_ERR_HIP;
        }
    }
    s->thread = std::thread([s] { s->run(); });
    *out = s;
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_server_create(int64_t arena_bytes, int32_t n_slots, int32_t max_batch_jobs, hk_server **out) {
    return create(arena_bytes, n_slots, max_batch_jobs, false, 0, 0.0, out);
}

int hk_server_create_simulated(int64_t arena_bytes, int32_t n_slots, int32_t max_batch_jobs, int64_t batch_fixed_ns,
                               double ns_per_site, hk_server **out) {
    return create(arena_bytes, n_slots, max_batch_jobs, true, batch_fixed_ns, ns_per_site, out);
}

int64_t hk_server_now_ns(void) { return now_ns(); }

int64_t hk_server_footprint(int32_t nx, int32_t ny, int32_t nz) {
    if (nx < 1 || ny < 1 || nz < 1) return HK_ERR_INVALID_ARG;
    const int64_t n = (int64_t)nx * ny * nz;
    if (n > INT32_MAX) return HK_ERR_TOO_LARGE;
    Geo g;
    const int rc = plan_lattice_ext(nx, ny, nz, 0u, &g);
    if (rc != HK_OK) return rc;
    int64_t lab, outb;
    output_bytes(n, &lab, &outb);
    return outb + batch_block_bytes(1, al(lattice_bytes(g)));
}

}  // extern "C"

namespace {

int submit(hk_server *s, const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
           int64_t arrival_ns, bool after, hipStream_t producer, uint64_t *ticket) {
    if (!s || !ticket || (!phi && !s->sim)) return HK_ERR_INVALID_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || periodic_mask > 7u) return HK_ERR_INVALID_ARG;
    const int64_t n = (int64_t)nx * ny * nz;
    if (n > INT32_MAX) return HK_ERR_TOO_LARGE;
    Request r;
    Geo g;
    const int rc = plan_lattice_ext(nx, ny, nz, periodic_mask, &g);
    if (rc != HK_OK) return rc;
    r.phi = phi;
    r.nx = nx, r.ny = ny, r.nz = nz;
    r.mask = periodic_mask;
    r.sites = n;
    r.ws_bytes = al(lattice_bytes(g));
    output_bytes(n, &r.lab_bytes, &r.out_bytes);
    r.arrival = arrival_ns > 0 ? arrival_ns : now_ns();
    // a request that can never fit alone is refused now
    if (r.out_bytes + batch_block_bytes(1, r.ws_bytes) > s->arena.size()) return HK_ERR_TOO_LARGE;
    bool wake;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->sim && after) {
            // phi is complete once the producer stream's present work is;
            // a stream with nothing pending needs no event
            const hipError_t q = hipStreamQuery(producer);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                r.ready = s->take_event();
                r.producer = producer;
                if (!r.ready || hipEventRecord(r.ready, producer) != hipSuccess) {
                    if (r.ready) s->event_pool.push_back(r.ready);
                    (void)hipGetLastError();
                    return HK_ERR_HIP;
                }
            } else if (q != hipSuccess) {
                (void)hipGetLastError();
                return HK_ERR_HIP;
            }
        }
        const uint64_t t = s->next_ticket++;
        s->reqs.emplace(t, r);
        // the scheduler waits without a deadline only on an empty queue;
        // otherwise it looks at the queue again within 20 us by itself
        wake = s->queue.empty();
        s->queue.push_back(t);
        ++s->submitted;
        *ticket = t;
    }
    if (wake) s->work_cv.notify_one();
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_server_submit(hk_server *s, const float *phi, int32_t nx, int32_t ny, int32_t nz, uint32_t periodic_mask,
                     int64_t arrival_ns, uint64_t *ticket) {
    return submit(s, phi, nx, ny, nz, periodic_mask, arrival_ns, false, nullptr, ticket);
}

int hk_server_submit_after(hk_server *s, const float *phi, int32_t nx, int32_t ny, int32_t nz,
                           uint32_t periodic_mask, int64_t arrival_ns, hipStream_t producer, uint64_t *ticket) {
    return submit(s, phi, nx, ny, nz, periodic_mask, arrival_ns, true, producer, ticket);
}

int hk_server_poll(hk_server *s, uint64_t ticket) {
    if (!s) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return HK_ERR_INVALID_ARG;
    if (it->second.state == State::Failed) return it->second.status;
    return it->second.state == State::Done ? 1 : 0;
}

int hk_server_wait(hk_server *s, uint64_t ticket, int64_t timeout_ns) {
    if (!s) return HK_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::nanoseconds(std::max<int64_t>(0, timeout_ns));
    for (;;) {
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return HK_ERR_INVALID_ARG;
        if (it->second.state == State::Done) return HK_OK;
        if (it->second.state == State::Failed) return it->second.status;
        if (s->done_cv.wait_until(lk, until) == std::cv_status::timeout) {
            it = s->reqs.find(ticket);
            if (it != s->reqs.end() && it->second.state == State::Done) return HK_OK;
            if (it != s->reqs.end() && it->second.state == State::Failed) return it->second.status;
            return HK_ERR_TIMEOUT;
        }
    }
}

int hk_server_drain(hk_server *s, int64_t timeout_ns) {
    if (!s) return HK_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::nanoseconds(std::max<int64_t>(0, timeout_ns));
    auto idle = [s] {
        if (!s->queue.empty()) return false;
        for (const Slot &sl : s->slots)
            if (sl.busy) return false;
        return true;
    };
    while (!idle())
        if (s->done_cv.wait_until(lk, until) == std::cv_status::timeout) return idle() ? HK_OK : HK_ERR_TIMEOUT;
    return HK_OK;
}

int hk_server_result(hk_server *s, uint64_t ticket, int32_t **labels, int64_t *n_clusters, int64_t **sizes,
                     int64_t *latency_ns) {
    if (!s) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return HK_ERR_INVALID_ARG;
    const Request &r = it->second;
    if (r.state == State::Failed) return r.status;
    if (r.state != State::Done) return HK_ERR_INVALID_ARG;
    // a simulated server has no arena memory: its pointers are the offsets
    // (computed as integers, since no object lies behind them)
    const uintptr_t at = (uintptr_t)s->base + (uintptr_t)r.out_off;
    if (labels) *labels = (int32_t *)at;
    if (sizes) *sizes = (int64_t *)(at + (uintptr_t)r.lab_bytes);
    if (n_clusters) *n_clusters = r.k;
    if (latency_ns) *latency_ns = r.done - r.arrival;
    return HK_OK;
}

int hk_server_release(hk_server *s, uint64_t ticket) {
    if (!s) return HK_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return HK_ERR_INVALID_ARG;
        Request &r = it->second;
        if (r.state == State::Running) return HK_ERR_INVALID_ARG;
        if (r.state == State::Pending) {
            s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
            if (r.ready) s->event_pool.push_back(r.ready);
        } else if (r.out_off >= 0) {
            s->arena.release(r.out_off, r.out_bytes);
        }
        s->reqs.erase(it);
    }
    s->work_cv.notify_one();
    return HK_OK;
}

int hk_server_read_stats(hk_server *s, hk_server_stats *out) {
    if (!s || !out) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->batches = s->batches;
    out->mean_batch_jobs = s->batches ? (double)s->batched_jobs / (double)s->batches : 0.0;
    out->sites_completed = s->sites_done;
    out->arena_bytes = s->arena.size();
    out->arena_in_use = s->arena.used();
    out->arena_peak = s->arena.peak();
    int64_t pending = 0, running = 0;
    for (const auto &kv : s->reqs) {
        pending += kv.second.state == State::Pending;
        running += kv.second.state == State::Running;
    }
    out->pending = pending;
    out->running = running;
    out->span_ns = s->last_done > s->first_launch ? s->last_done - s->first_launch : 0;
    std::vector<int64_t> v = s->lat;
    out->latency_samples = (int64_t)v.size();
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto rank = [&](double q) {
            // nearest rank: the smallest sample with at least q of the samples <= it
            int64_t r = (int64_t)std::ceil(q * (double)v.size());
            r = std::min<int64_t>(std::max<int64_t>(r, 1), (int64_t)v.size());
            return v[(size_t)(r - 1)];
        };
        double sum = 0.0;
        for (int64_t x : v) sum += (double)x;
        out->latency_p50_ns = rank(0.50);
        out->latency_p99_ns = rank(0.99);
        out->latency_max_ns = v.back();
        out->latency_mean_ns = sum / (double)v.size();
    }
    return HK_OK;
}

int hk_server_reset_stats(hk_server *s) {
    if (!s) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->reset_stats();
    return HK_OK;
}

int hk_server_destroy(hk_server *s) {
    if (!s) return HK_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->work_cv.notify_all();
    if (s->thread.joinable()) s->thread.join();
    if (!s->sim) {
        for (Slot &sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        for (auto &kv : s->reqs)
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
        for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
        if (s->base) (void)hipFree(s->base);
    }
    delete s;
    return HK_OK;
}

int hk_server_sim_fail(hk_server *s, uint64_t ticket, int32_t status) {
    if (!s || !s->sim || status >= 0) return HK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != State::Pending) return HK_ERR_INVALID_ARG;
    it->second.sim_fail = status;
    return HK_OK;
}

}  // extern "C"
