// Continuous-batching server for snapshot-vs-reference IQA requests.
//
// Reference images stay resident in device memory.  Each request names a
// reference, a tile size and a snapshot (already on the device, or in pinned
// host memory that the server copies in), plus device buffers for its IQA
// matrices.  A scheduler thread admits requests in arrival order while the
// bytes held by admitted, unfinished requests stay under an HBM budget, packs
// everything admitted into one launch of the persistent batched kernel
// whenever one of its `streams` launch slots is free, and retires a batch when
// its completion word says so.  Requests that arrive while batches run are
// admitted as budget and slots free up and go out with the next launch, so
// batches overlap on the device (one stream per slot).
//
// Completion: after each batch the slot's stream runs a one-thread kernel that
// stores the batch's sequence number into a word of pinned host memory, and
// the scheduler polls that word.  Stream order makes the store follow the
// batch (and any snapshot copies before it).  A HIP event would do the same
// job, but recording one has a long host-side latency tail (tens of
// microseconds at the 99th percentile) and its completion is seen later.
//
// A request's results do not depend on what it is batched with: each pair in
// a batch is reduced by its own waves, in a fixed order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "iqa.h"
#include "iqa_internal.h"

namespace iqa_srv {

// Publishes a finished batch: stores its sequence number into the slot's
// completion word (system scope, so the host sees it without any HIP call).
__global__ void publish_kernel(uint32_t *word, uint32_t seq) {
    if (threadIdx.x == 0) __hip_atomic_store(word, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace iqa_srv

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Ref {
    const float *ptr;
    int64_t N;
};

struct Pending {
    iqa_request req;
    int64_t t_submit;
    int64_t t_admit = 0;
    int64_t cost = 0;
};

// One launch slot: its stream, completion word, pinned descriptor staging,
// device descriptor table and (for host snapshots) a device snapshot arena.
struct Slot {
    hipStream_t stream = nullptr;
    uint32_t *word_host = nullptr;   // pinned, host-coherent completion word
    uint32_t *word_dev = nullptr;    // the same word as the device sees it
    uint32_t seq = 0;                // number of the batch in flight
    int64_t t_checked = 0;           // last time the stream was asked for errors
    void *desc_host = nullptr;
    void *desc_dev = nullptr;
    float *arena = nullptr;      // device, for snapshots copied from the host
    int64_t arena_bytes = 0;
    bool busy = false;
    int64_t t_launch = 0;
    int64_t bytes = 0;           // budget held by this batch
    int64_t dry_due = 0;         // dry run: when the simulated batch completes
    std::vector<Pending> reqs;
};

hipError_t launch_publish(const Slot &s) {
    uint32_t *word = s.word_dev;
    uint32_t seq = s.seq;
    void *args[] = {&word, &seq};
    return hipLaunchKernel(reinterpret_cast<const void *>(&iqa_srv::publish_kernel), dim3(1),
                           dim3(64), args, 0, s.stream);
}

// How long a batch may run before the scheduler also asks its stream whether
// it failed (a failed batch never publishes).
constexpr int64_t kErrorCheckNs = 1000000;

// The first launch of a kernel in a process, and the first work on a new
// stream, can hold the device for milliseconds; left to the first requests,
// that shows as a burst of millisecond latencies at the start of a server's
// life.  At creation the server therefore runs every launch form it can use
// once, on a tiny zero pair, and waits for it: the batch kernel with 1, 4 and
// IQA_BATCH_INLINE_MAX descriptors in its arguments and with a descriptor
// table (as far as max_batch allows), and the publishing kernel on every slot
// stream (storing 0, the word's initial value).  Returns the first HIP error.
hipError_t warm_up(std::vector<Slot> &slots, const iqa_server_opts &o) {
    constexpr int64_t kN = 32;   // one 32 x 32 tile per pair
    constexpr int64_t kPairs = IQA_BATCH_INLINE_MAX + 1;
    const int64_t img = kN * kN;
    float *buf = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&buf),
                             (size_t)(img + 2 * kPairs) * sizeof(float));
    if (e != hipSuccess) return e;
    Slot &s0 = slots[0];
    e = hipMemsetAsync(buf, 0, (size_t)img * sizeof(float), s0.stream);
    const int64_t counts[] = {1, 4, IQA_BATCH_INLINE_MAX, IQA_BATCH_INLINE_MAX + 1};
    int64_t prev = 0;
    for (int64_t c : counts) {
        c = std::min<int64_t>(c, o.max_batch);
        if (e != hipSuccess || c == prev) continue;
        prev = c;
        std::vector<iqa_pair> pairs((size_t)c);
        for (int64_t i = 0; i < c; ++i)
            pairs[(size_t)i] = iqa_pair{buf, buf, kN, kN, o.D, o.C1, o.C2, o.C,
                                        buf + img + 2 * i, buf + img + 2 * i + 1, nullptr};
        int64_t units = 0;
        // Constants a request could not use either: nothing to warm up.
        if (iqa::describe_pairs(pairs.data(), c, s0.desc_host, &units, IQA_TUNE_SERVE) != IQA_OK)
            break;
        iqa_status st;
        if (c <= IQA_BATCH_INLINE_MAX) {
            st = iqa_tiles_batched_inline(s0.desc_host, c, units, o.waves, s0.stream);
        } else {
            e = hipMemcpyAsync(s0.desc_dev, s0.desc_host, (size_t)c * IQA_BATCH_DESC_BYTES,
                               hipMemcpyHostToDevice, s0.stream);
            st = e == hipSuccess ? iqa_tiles_batched(s0.desc_dev, c, units, o.waves, s0.stream)
                                 : IQA_OK;
        }
        if (st == IQA_ERR_HIP) {
            e = (hipError_t)iqa_last_hip_error();
            if (e == hipSuccess) e = hipErrorUnknown;
        } else if (st != IQA_OK) {
            break;   // a launch the scheduler would refuse the same way
        }
    }
    for (Slot &s : slots)
        if (e == hipSuccess) e = launch_publish(s);
    for (Slot &s : slots) {
        const hipError_t w = hipStreamSynchronize(s.stream);
        if (e == hipSuccess) e = w;
    }
    const hipError_t f = hipFree(buf);
    return e == hipSuccess ? f : e;
}

}  // namespace

struct iqa_server {
    iqa_server_opts opts{};
    int device = 0;
    // Dry run: schedule exactly as below but launch nothing; a batch of b
    // bytes completes dry_fixed_ns + b / dry_bytes_per_ns after its launch.
    bool dry = false;
    int64_t dry_fixed_ns = 0;
    double dry_bytes_per_ns = 1.0;
    std::vector<Ref> refs;
    std::vector<Slot> slots;

    std::mutex mu;               // guards intake, done, counters below
    std::condition_variable cv;  // wakes the scheduler
    std::condition_variable cv_done;
    std::deque<Pending> intake;
    std::deque<iqa_completion> done;
    int64_t submitted = 0, completed = 0;
    int64_t in_flight_bytes = 0, peak_in_flight_bytes = 0;
    int64_t batches = 0, max_batch_seen = 0, rejected = 0;
    // Set under mu; also read without it by the scheduler loop.
    std::atomic<bool> stop{false};
    // intake.size(), published under mu, so that the scheduler loop can see
    // new work without taking the lock (a spinning loop that takes mu on every
    // pass delays the submitting threads).
    std::atomic<int64_t> intake_n{0};
    // done.size(), published under mu, so that a poll with nothing to return
    // (a caller polling in a loop) does not take the lock.
    std::atomic<int64_t> done_n{0};
    // Written by the scheduler thread, read by get_stats from any thread.
    std::atomic<int> last_hip_error{0};

    std::deque<Pending> pending;  // scheduler-owned: admitted order
    std::thread worker;

    void run();
    bool launch(Slot &s, std::vector<Pending> &batch);
    void retire(Slot &s, int status);
};

namespace {

int64_t request_cost(const iqa_server &sv, const iqa_request &r) {
    const int64_t N = sv.refs[r.ref_id].N;
    const int64_t ns = N / r.NT;
    // the snapshot the request holds plus its output matrices
    return 4 * N * N + 8 * ns * ns + (r.sums ? 16 * ns * ns : 0);
}

}  // namespace

bool iqa_server::launch(Slot &s, std::vector<Pending> &batch) {
    if (dry) {
        int64_t bytes = 0;
        for (const Pending &p : batch) bytes += 8 * refs[p.req.ref_id].N * refs[p.req.ref_id].N;
        s.reqs.swap(batch);
        s.busy = true;
        s.t_launch = now_ns();
        s.dry_due = s.t_launch + dry_fixed_ns + (int64_t)((double)bytes / dry_bytes_per_ns);
        return true;
    }
    std::vector<iqa_pair> pairs(batch.size());
    int64_t arena_off = 0;
    bool ok = true;
    // The batch's stream waits for every request's ready event (each distinct
    // event once) before anything reads a snapshot or writes an output.
    void *waited = nullptr;
    for (size_t i = 0; i < batch.size() && ok; ++i) {
        void *ev = batch[i].req.ready_event;
        if (!ev || ev == waited) continue;
        hipError_t e = hipStreamWaitEvent(s.stream, static_cast<hipEvent_t>(ev), 0);
        if (e != hipSuccess) {
            last_hip_error = (int)e;
            ok = false;
        }
        waited = ev;
    }
    for (size_t i = 0; i < batch.size(); ++i) {
        const iqa_request &r = batch[i].req;
        const Ref &ref = refs[r.ref_id];
        const float *snap = r.snapshot_dev;
        if (!snap) {
            // Copy the host snapshot into this slot's arena (16-byte aligned).
            const int64_t bytes = 4 * ref.N * ref.N;
            float *dst = reinterpret_cast<float *>(reinterpret_cast<char *>(s.arena) + arena_off);
            arena_off += (bytes + 255) & ~int64_t(255);
            hipError_t e = hipMemcpyAsync(dst, r.snapshot_host, bytes, hipMemcpyHostToDevice,
                                          s.stream);
            if (e != hipSuccess) {
                last_hip_error = (int)e;
                ok = false;
            }
            snap = dst;
        }
        pairs[i] = iqa_pair{snap, ref.ptr, ref.N, r.NT, opts.D, opts.C1, opts.C2, opts.C,
                            r.lisi, r.auglisi, r.sums};
    }
    int64_t units = 0;
    if (ok && iqa::describe_pairs(pairs.data(), (int64_t)pairs.size(), s.desc_host, &units,
                                  IQA_TUNE_SERVE) != IQA_OK)
        ok = false;
    // Small batches carry their descriptors in the kernel arguments (one
    // enqueue); larger ones copy the table to the slot's device buffer first.
    const bool inl = pairs.size() <= (size_t)IQA_BATCH_INLINE_MAX;
    if (ok && !inl) {
        hipError_t e = hipMemcpyAsync(s.desc_dev, s.desc_host,
                                      pairs.size() * IQA_BATCH_DESC_BYTES,
                                      hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) {
            last_hip_error = (int)e;
            ok = false;
        }
    }
    if (ok) {
        const iqa_status st =
            inl ? iqa_tiles_batched_inline(s.desc_host, (int64_t)pairs.size(), units, opts.waves,
                                           s.stream)
                : iqa_tiles_batched(s.desc_dev, (int64_t)pairs.size(), units, opts.waves,
                                    s.stream);
        if (st != IQA_OK) {
            last_hip_error = iqa_last_hip_error();
            ok = false;
        }
    }
    if (ok) {
        s.seq += 1;
        hipError_t e = launch_publish(s);
        if (e != hipSuccess) {
            last_hip_error = (int)e;
            ok = false;
        }
    }
    s.reqs.swap(batch);
    s.busy = true;
    s.t_launch = now_ns();
    s.t_checked = s.t_launch;
    return ok;
}

void iqa_server::retire(Slot &s, int status) {
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lock(mu);
    for (const Pending &p : s.reqs) {
        iqa_completion c{};
        c.tag = p.req.tag;
        c.status = status;
        c.t_submit_ns = p.t_submit;
        c.t_admit_ns = p.t_admit;
        c.t_launch_ns = s.t_launch;
        c.t_done_ns = t;
        done.push_back(c);
    }
    done_n.store((int64_t)done.size(), std::memory_order_release);
    completed += (int64_t)s.reqs.size();
    in_flight_bytes -= s.bytes;
    s.reqs.clear();
    s.bytes = 0;
    s.busy = false;
    cv_done.notify_all();
}

void iqa_server::run() {
    if (!dry) (void)hipSetDevice(device);
    const int64_t budget = opts.hbm_budget_bytes;
    std::vector<Pending> batch;
    int64_t last_active = now_ns();
    while (true) {
        bool idle = true;
        if (intake_n.load(std::memory_order_acquire) > 0) {
            std::lock_guard<std::mutex> lock(mu);
            while (!intake.empty()) {
                pending.push_back(intake.front());
                intake.pop_front();
            }
            intake_n.store(0, std::memory_order_relaxed);
            idle = false;
        }
        if (stop.load(std::memory_order_acquire) && pending.empty()) {
            bool any_busy = false;
            for (const Slot &s : slots) any_busy |= s.busy;
            if (!any_busy) {
                // submit refuses new work once stop is set (under mu), so an
                // empty intake seen under mu stays empty.
                std::lock_guard<std::mutex> lock(mu);
                if (intake.empty()) break;
                continue;
            }
        }
        // Retire finished batches.
        for (Slot &s : slots) {
            if (!s.busy) continue;
            if (dry) {
                if (now_ns() >= s.dry_due) {
                    retire(s, IQA_OK);
                    idle = false;
                }
                continue;
            }
            if (__atomic_load_n(s.word_host, __ATOMIC_ACQUIRE) == s.seq) {
                retire(s, IQA_OK);
                idle = false;
                continue;
            }
            const int64_t t = now_ns();
            if (t - s.t_checked < kErrorCheckNs) continue;
            s.t_checked = t;
            const hipError_t q = hipStreamQuery(s.stream);
            if (q == hipErrorNotReady) continue;
            // The stream has finished (or failed): its publish store, if it
            // ran, is visible now.
            if (q == hipSuccess && __atomic_load_n(s.word_host, __ATOMIC_ACQUIRE) == s.seq) {
                retire(s, IQA_OK);
            } else {
                last_hip_error = q == hipSuccess ? (int)hipErrorUnknown : (int)q;
                retire(s, IQA_ERR_HIP);
            }
            idle = false;
        }
        // Launch into a free slot everything the budget admits, in order.
        for (Slot &s : slots) {
            if (s.busy || pending.empty()) continue;
            batch.clear();
            int64_t held, arena_used = 0;
            {
                std::lock_guard<std::mutex> lock(mu);
                held = in_flight_bytes;
            }
            int64_t add = 0;
            while (!pending.empty() && (int64_t)batch.size() < opts.max_batch) {
                Pending &p = pending.front();
                const int64_t N = refs[p.req.ref_id].N;
                const int64_t snap = p.req.snapshot_dev ? 0 : ((4 * N * N + 255) & ~int64_t(255));
                if (held + add + p.cost > budget) break;
                if (arena_used + snap > s.arena_bytes) break;
                add += p.cost;
                arena_used += snap;
                p.t_admit = now_ns();
                batch.push_back(p);
                pending.pop_front();
            }
            if (batch.empty()) break;
            {
                std::lock_guard<std::mutex> lock(mu);
                in_flight_bytes += add;
                peak_in_flight_bytes = std::max(peak_in_flight_bytes, in_flight_bytes);
                batches += 1;
                max_batch_seen = std::max<int64_t>(max_batch_seen, (int64_t)batch.size());
            }
            s.bytes = add;
            if (!launch(s, batch)) {
                // Let whatever was enqueued finish before the slot is reused.
                if (!dry) (void)hipStreamSynchronize(s.stream);
                retire(s, IQA_ERR_HIP);
            }
            idle = false;
        }
        if (!idle) {
            last_active = now_ns();
        } else {
            bool any_busy = false;
            for (const Slot &s : slots) any_busy |= s.busy;
            if (any_busy || now_ns() - last_active < opts.idle_spin_ns) {
                // Poll the completion words (or, for idle_spin_ns after the
                // last work, the intake count) without sleeping and without
                // the lock: a wake-up from the condition variable costs tens
                // of microseconds.
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lock(mu);
                if (intake.empty() && !stop.load(std::memory_order_relaxed))
                    cv.wait_for(lock, std::chrono::milliseconds(1));
            }
        }
    }
}

extern "C" {

static iqa_status check_opts(const iqa_server_opts *opts) {
    if (opts->streams < 1 || opts->streams > 16 || opts->max_batch < 1 ||
        opts->max_batch > (1 << 20) || opts->hbm_budget_bytes <= 0 ||
        opts->host_arena_bytes < 0)
        return IQA_ERR_CONFIG;
    if (opts->waves != 0 && (opts->waves < 4 || opts->waves % 4 != 0)) return IQA_ERR_CONFIG;
    if (opts->idle_spin_ns < 0 || opts->idle_spin_ns > 1000000000) return IQA_ERR_CONFIG;
    return IQA_OK;
}

iqa_status iqa_server_create(const iqa_server_opts *opts, iqa_server **out) {
    if (!opts || !out) return IQA_ERR_NULL;
    iqa_status st = check_opts(opts);
    if (st != IQA_OK) return st;
    auto *sv = new iqa_server();
    sv->opts = *opts;
    if (sv->opts.waves == 0) sv->opts.waves = iqa_batch_default_waves();
    hipError_t e = hipGetDevice(&sv->device);
    sv->slots.resize(opts->streams);
    for (Slot &s : sv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&s.word_host), 64,
                              hipHostMallocCoherent | hipHostMallocMapped);
        if (e == hipSuccess) {
            *s.word_host = 0;
            e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s.word_dev), s.word_host, 0);
        }
        if (e == hipSuccess)
            e = hipHostMalloc(&s.desc_host, (size_t)opts->max_batch * IQA_BATCH_DESC_BYTES,
                              hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc(&s.desc_dev, (size_t)opts->max_batch * IQA_BATCH_DESC_BYTES);
        if (e == hipSuccess && opts->host_arena_bytes > 0) {
            e = hipMalloc(reinterpret_cast<void **>(&s.arena), (size_t)opts->host_arena_bytes);
            s.arena_bytes = opts->host_arena_bytes;
        }
    }
    if (e == hipSuccess) e = warm_up(sv->slots, sv->opts);
    if (e != hipSuccess) {
        iqa_server_destroy(sv);
        return IQA_ERR_HIP;
    }
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    return IQA_OK;
}

iqa_status iqa_server_create_dry(const iqa_server_opts *opts, int64_t fixed_ns,
                                 double bytes_per_ns, iqa_server **out) {
    if (!opts || !out) return IQA_ERR_NULL;
    iqa_status st = check_opts(opts);
    if (st != IQA_OK) return st;
    if (fixed_ns < 0 || !(bytes_per_ns > 0.0)) return IQA_ERR_CONFIG;
    auto *sv = new iqa_server();
    sv->opts = *opts;
    sv->dry = true;
    sv->dry_fixed_ns = fixed_ns;
    sv->dry_bytes_per_ns = bytes_per_ns;
    sv->slots.resize(opts->streams);
    for (Slot &s : sv->slots) s.arena_bytes = opts->host_arena_bytes;
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    return IQA_OK;
}

iqa_status iqa_server_add_reference(iqa_server *sv, const float *ref, int64_t N,
                                    int32_t *ref_id) {
    if (!sv || !ref || !ref_id) return IQA_ERR_NULL;
    if (N <= 0 || N > IQA_MAX_N) return IQA_ERR_SHAPE;
    if ((reinterpret_cast<uintptr_t>(ref) % 16) != 0) return IQA_ERR_ALIGN;
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->submitted > 0) return IQA_ERR_CONFIG;   // references are fixed once serving
    sv->refs.push_back(Ref{ref, N});
    *ref_id = (int32_t)sv->refs.size() - 1;
    return IQA_OK;
}

iqa_status iqa_server_submit(iqa_server *sv, const iqa_request *reqs, int64_t count) {
    if (!sv || !reqs) return IQA_ERR_NULL;
    if (count < 0) return IQA_ERR_SHAPE;
    const int64_t t = now_ns();
    // Validation reads the reference table, so it runs under the lock that
    // add_reference takes: a first submit cannot race a late add_reference.
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->stop) return IQA_ERR_CONFIG;
    int64_t rejected = 0;
    for (int64_t i = 0; i < count; ++i) {
        const iqa_request &r = reqs[i];
        int st = IQA_OK;
        if (r.ref_id < 0 || r.ref_id >= (int32_t)sv->refs.size()) {
            st = IQA_ERR_CONFIG;
        } else {
            const int64_t N = sv->refs[r.ref_id].N;
            if (r.NT <= 0 || N % r.NT != 0 || r.NT % 4 != 0) st = IQA_ERR_SHAPE;
            else if (!r.snapshot_dev == !r.snapshot_host) st = IQA_ERR_NULL;
            else if (!r.lisi && !r.auglisi && !r.sums) st = IQA_ERR_NULL;
            else if (r.snapshot_dev && (reinterpret_cast<uintptr_t>(r.snapshot_dev) % 16))
                st = IQA_ERR_ALIGN;
            else if (request_cost(*sv, r) > sv->opts.hbm_budget_bytes) st = IQA_ERR_BUDGET;
            else if (r.snapshot_host &&
                     ((4 * N * N + 255) & ~int64_t(255)) > sv->opts.host_arena_bytes)
                st = IQA_ERR_BUDGET;
        }
        if (st != IQA_OK) {
            iqa_completion c{};
            c.tag = r.tag;
            c.status = st;
            c.t_submit_ns = c.t_admit_ns = c.t_launch_ns = c.t_done_ns = c.t_poll_ns = t;
            sv->done.push_back(c);
            ++rejected;
            continue;
        }
        Pending p;
        p.req = r;
        p.t_submit = t;
        p.cost = request_cost(*sv, r);
        sv->intake.push_back(p);
    }
    sv->intake_n.store((int64_t)sv->intake.size(), std::memory_order_release);
    sv->done_n.store((int64_t)sv->done.size(), std::memory_order_release);
    sv->submitted += count;
    sv->completed += rejected;
    sv->rejected += rejected;
    sv->cv.notify_one();
    sv->cv_done.notify_all();
    return IQA_OK;
}

int64_t iqa_server_poll(iqa_server *sv, iqa_completion *out, int64_t max) {
    if (!sv || !out || max <= 0) return 0;
    if (sv->done_n.load(std::memory_order_acquire) == 0) return 0;
    int64_t n = 0;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        while (n < max && !sv->done.empty()) {
            out[n++] = sv->done.front();
            sv->done.pop_front();
        }
        sv->done_n.store((int64_t)sv->done.size(), std::memory_order_relaxed);
    }
    const int64_t t = now_ns();
    for (int64_t i = 0; i < n; ++i) out[i].t_poll_ns = t;
    return n;
}

iqa_status iqa_server_drain(iqa_server *sv, int64_t timeout_ms) {
    if (!sv) return IQA_ERR_NULL;
    std::unique_lock<std::mutex> lock(sv->mu);
    const bool ok = sv->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms),
                                         [sv] { return sv->completed == sv->submitted; });
    return ok ? IQA_OK : IQA_ERR_TIMEOUT;
}

iqa_status iqa_server_get_stats(iqa_server *sv, iqa_server_stats *st) {
    if (!sv || !st) return IQA_ERR_NULL;
    std::lock_guard<std::mutex> lock(sv->mu);
    st->submitted = sv->submitted;
    st->completed = sv->completed;
    st->rejected = sv->rejected;
    st->batches = sv->batches;
    st->max_batch = sv->max_batch_seen;
    st->in_flight_bytes = sv->in_flight_bytes;
    st->peak_in_flight_bytes = sv->peak_in_flight_bytes;
    st->last_hip_error = sv->last_hip_error.load();
    return IQA_OK;
}

iqa_status iqa_server_replay(iqa_server *sv, const iqa_request *reqs,
                             const int64_t *arrival_ns, int64_t count, iqa_completion *out,
                             int64_t timeout_ms) {
    if (!sv || !reqs || !arrival_ns || !out) return IQA_ERR_NULL;
    if (count < 0) return IQA_ERR_SHAPE;
    for (int64_t i = 1; i < count; ++i)
        if (arrival_ns[i] < arrival_ns[i - 1]) return IQA_ERR_CONFIG;
    // Open loop: an arrival thread submits request i at start + arrival_ns[i]
    // whatever the state of the server; this thread collects completions.
    const int64_t t0 = now_ns() + 1000000;   // 1 ms to get going
    std::atomic<bool> abort{false};
    std::thread arrivals([&] {
        for (int64_t i = 0; i < count && !abort.load(); ++i) {
            const int64_t due = t0 + arrival_ns[i];
            while (now_ns() < due) {
                if (due - now_ns() > 200000) std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
            iqa_server_submit(sv, &reqs[i], 1);
        }
    });
    std::vector<iqa_completion> got;
    got.reserve(count);
    std::vector<iqa_completion> buf(4096);
    const int64_t deadline = now_ns() + timeout_ms * 1000000;
    iqa_status st = IQA_OK;
    while ((int64_t)got.size() < count) {
        const int64_t n = iqa_server_poll(sv, buf.data(), (int64_t)buf.size());
        for (int64_t i = 0; i < n; ++i) got.push_back(buf[i]);
        if (n == 0) {
            if (now_ns() > deadline) {
                st = IQA_ERR_TIMEOUT;
                abort.store(true);
                break;
            }
            std::this_thread::yield();
        }
    }
    arrivals.join();
    // Completion order; times relative to the start of the trace.
    for (int64_t i = 0; i < (int64_t)got.size() && i < count; ++i) {
        out[i] = got[i];
        out[i].t_submit_ns -= t0;
        out[i].t_admit_ns -= t0;
        out[i].t_launch_ns -= t0;
        out[i].t_done_ns -= t0;
        out[i].t_poll_ns -= t0;
    }
    return st;
}

iqa_status iqa_server_destroy(iqa_server *sv) {
    if (!sv) return IQA_ERR_NULL;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.word_host) (void)hipHostFree(s.word_host);
        if (s.desc_host) (void)hipHostFree(s.desc_host);
        if (s.desc_dev) (void)hipFree(s.desc_dev);
        if (s.arena) (void)hipFree(s.arena);
    }
    delete sv;
    return IQA_OK;
}

}  // extern "C"
