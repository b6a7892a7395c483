// Serving: continuous batching of decode requests over the fused batch path.
//
// One scheduler thread per server.  Requests wait in a FIFO queue; whenever
// one of the launch slots (each with its own stream) is free and the device
// arena has room, the scheduler takes the longest prefix of the queue that
// fits the group cap and the free memory, packs the group's LLRs contiguously
// in pinned host staging, and enqueues on the slot's stream: a copy kernel that
// moves them into the device arena, ldpc_decode_batch over the group's jobs
// (which writes bits, iteration counts and posteriors straight into pinned
// host memory), and an event.  Groups admitted while
// others are still running use other slots, so their kernels overlap with the
// running ones on the device.  Completed slots are reaped by polling their
// events; results are copied into the requesters' buffers and the memory is
// returned to the arena.  The lock is held only to move requests between the
// queue and the slots: the staging copies, launches and result copies run
// without it, so a large group never holds up submitters.  Arithmetic is per
// frame, so a request's result does not depend on what it was batched with.
#include <sys/resource.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ldpc_internal.h"

namespace {

int64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return static_cast<int64_t>(ts.tv_sec) * 1000000000LL + ts.tv_nsec;
}

int64_t thread_cpu_ns()
{
    timespec ts;
    clock_gettime(CLOCK_THREAD_CPUTIME_ID, &ts);
    return static_cast<int64_t>(ts.tv_sec) * 1000000000LL + ts.tv_nsec;
}

// Scheduler steps slower than kTraceStepNs are recorded when the environment
// variable LDPC_SERVER_TRACE names a file (written when the server is
// destroyed): where the step's time went, the thread's CPU time in it and
// its context switches, to tell a blocked or preempted thread from work.
constexpr int64_t kTraceStepNs = 500000;
struct StepTrace {
    int64_t start_ns, wall_ns, cpu_ns, sleep_ns;  // sleep_ns: the wait before this step
    int64_t copy_ns, launch_ns, query_ns;         // longest of each inside the step
    long nvcsw, nivcsw;                           // voluntary / involuntary context switches in the step
};

// First-fit allocator of contiguous ranges in [0, capacity).
class RangeAlloc {
  public:
    explicit RangeAlloc(int64_t cap = 0) : cap_(cap)
    {
        if (cap > 0)
            free_.push_back({0, cap});
    }
    int64_t alloc(int64_t len)
    {
        for (size_t i = 0; i < free_.size(); ++i)
            if (free_[i].second >= len) {
                const int64_t b = free_[i].first;
                free_[i].first += len;
                free_[i].second -= len;
                if (free_[i].second == 0)
                    free_.erase(free_.begin() + static_cast<long>(i));
                return b;
            }
        return -1;
    }
    void release(int64_t begin, int64_t len)
    {
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(begin, int64_t(0)));
        it = free_.insert(it, {begin, len});
        size_t i = static_cast<size_t>(it - free_.begin());
        if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
            free_[i].second += free_[i + 1].second;
            free_.erase(free_.begin() + static_cast<long>(i) + 1);
        }
        if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
            free_[i - 1].second += free_[i].second;
            free_.erase(free_.begin() + static_cast<long>(i));
        }
    }
    int64_t capacity() const { return cap_; }

  private:
    int64_t cap_;
    std::vector<std::pair<int64_t, int64_t>> free_;  // (begin, length), sorted by begin
};

// LLR ranges are kept in multiples of 4 elements so that every range starts
// 16-byte aligned, as the copy kernel needs.
inline int64_t align4(int64_t e) { return (e + 3) & ~int64_t(3); }

// Workgroups of the staging copy (pinned host -> device arena): enough to
// keep the host link busy, few enough that the decode kernels of the other
// slots keep their compute units while it runs.
constexpr int32_t kLinkCopyBlocks = 64;

// Host copies of one group (LLRs into staging, results out of it), shared
// with helper threads when the group is large: one thread copies about
// 10 GB/s, and near capacity the next group's admission waits on these copies
// (the tail latency grows several-fold without the helpers).  The copy is cut
// into chunks that the calling (scheduler) thread and the helpers claim one at
// a time, so the caller never waits for a helper that has not started: a
// helper that wakes late (waking a sleeping thread has been seen to take
// milliseconds) finds the chunks taken, and the caller waits only for chunks
// already being copied.  Destinations are disjoint, so chunks are independent.
// Only the scheduler calls run().
class CopyPool {
  public:
    struct Item {
        void *dst;
        const void *src;
        size_t bytes;
    };
    static constexpr size_t kParallelBytes = 1 << 20;  // smaller groups are copied by the caller alone
    static constexpr size_t kChunkBytes = 64 << 10;

    explicit CopyPool(int helpers)
    {
        try {
            for (int i = 0; i < helpers; ++i)
                threads_.emplace_back([this] { loop(); });
        } catch (...) {
            shut_down();  // helpers started so far must be joined before the members go
            throw;
        }
    }
    ~CopyPool() { shut_down(); }

    void run(const std::vector<Item> &items)
    {
        size_t total = 0;
        for (const Item &it : items)
            total += it.bytes;
        if (threads_.empty() || total < kParallelBytes) {
            for (const Item &it : items)
                if (it.bytes)
                    std::memcpy(it.dst, it.src, it.bytes);
            return;
        }
        // No helper reads chunks_ now: the previous run ended with every
        // chunk claimed and copied.
        chunks_.clear();
        for (const Item &it : items)
            for (size_t off = 0; off < it.bytes; off += kChunkBytes)
                chunks_.push_back({static_cast<char *>(it.dst) + off, static_cast<const char *>(it.src) + off,
                                   std::min(kChunkBytes, it.bytes - off)});
        std::unique_lock<std::mutex> lk(mu_);
        next_ = 0;
        count_ = pending_ = chunks_.size();
        lk.unlock();
        go_.notify_all();
        lk.lock();
        copy_claimed(lk);
        done_.wait(lk, [&] { return pending_ == 0; });  // chunks helpers are copying right now
    }

  private:
    // Claims and copies chunks until none is left (called and returns with lk held).
    void copy_claimed(std::unique_lock<std::mutex> &lk)
    {
        while (next_ < count_) {
            const Item &c = chunks_[next_++];
            lk.unlock();
            std::memcpy(c.dst, c.src, c.bytes);
            lk.lock();
            if (--pending_ == 0)
                done_.notify_one();
        }
    }

    void shut_down()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        go_.notify_all();
        for (std::thread &t : threads_)
            t.join();
        threads_.clear();
    }

    void loop()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            go_.wait(lk, [&] { return stop_ || next_ < count_; });
            if (stop_)
                return;
            copy_claimed(lk);
        }
    }

    std::vector<std::thread> threads_;
    std::vector<Item> chunks_;  // written by run() only while no chunk is claimable
    std::mutex mu_;
    std::condition_variable go_, done_;
    size_t next_ = 0, count_ = 0, pending_ = 0;  // next chunk to claim, chunks, chunks not yet copied
    bool stop_ = false;
};

enum ReqState { kQueued = 0, kInFlight = 1, kDone = 2, kCancelled = 3 };

struct Request {
    uint64_t ticket = 0;
    int32_t code_id = 0, frames = 0, max_iter = 0;
    uint32_t flags = 0;
    const float *llr = nullptr;
    uint8_t *bits = nullptr;
    int32_t *iters = nullptr;
    float *post = nullptr;
    int64_t arrival_ns = 0, done_ns = 0;
    // scheduler milestones, for the slowest request's latency breakdown
    int64_t submit_ns = 0, admit_ns = 0, launch_ns = 0, seen_ns = 0;
    int state = kQueued;
    int64_t elem_off = 0, frame_off = 0;  // offsets inside the group's ranges
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    int64_t elem_begin = 0, elem_len = 0, frame_begin = 0, frame_len = 0;
    bool want_post = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

}  // namespace

struct ldpc_server_s {
    int device = 0;
    std::vector<ldpc_code> codes;
    std::vector<int32_t> code_n;
    int32_t max_group_frames = 0, max_queue = 0;
    // device arena of LLRs; pinned host memory for staged LLRs and results,
    // by its host (h_) and device (dh_) addresses; all share element offsets
    float *d_llr = nullptr;
    float *h_llr = nullptr, *h_post = nullptr, *dh_llr = nullptr, *dh_post = nullptr;
    uint8_t *h_bits = nullptr, *dh_bits = nullptr;
    int32_t *h_iters = nullptr, *dh_iters = nullptr;
    RangeAlloc elems, frames;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::atomic<uint64_t> submits{0};  // requests queued so far (read by the polling scheduler without the lock)
    std::deque<Request *> queue;
    // request of ticket t at by_ticket[t - 1]: tickets are consecutive, and a
    // deque grows in fixed blocks (no rehash or bulk move under the lock)
    std::deque<Request *> by_ticket;
    Request *find_ticket(uint64_t t) const
    {
        return t >= 1 && t <= by_ticket.size() ? by_ticket[static_cast<size_t>(t - 1)] : nullptr;
    }
    uint64_t next_ticket = 1;
    bool stop = false;
    bool broken = false;  // the scheduler hit a host allocation failure: requests fail from then on
    std::thread sched;
    std::unique_ptr<CopyPool> copies;  // used by the scheduler thread only
    std::vector<CopyPool::Item> copy_items;
    std::vector<ldpc_job> jobs;

    // statistics (guarded by mu)
    ldpc_server_stats st{};
    std::deque<double> lat_ms;  // grows in fixed blocks: no bulk move under the lock
    int64_t group_frames_sum = 0;
    double worst_ms = -1.0;     // latency of the request behind st.worst_*
    // slow-step trace (see StepTrace); the step_* maxima cover the current step
    std::string trace_path;
    std::vector<StepTrace> trace;
    int64_t step_copy_ns = 0, step_launch_ns = 0, step_query_ns = 0, t_created = 0;

    void run();
    void schedule(std::unique_lock<std::mutex> &lk);
    void fail_request(Request *r, int64_t t);
    void fail_everything(std::unique_lock<std::mutex> &lk);
    bool reap(std::unique_lock<std::mutex> &lk);
    bool admit(std::unique_lock<std::mutex> &lk);
    void free_all();
};

bool ldpc_server_s::reap(std::unique_lock<std::mutex> &lk)
{
    bool any = false;
    for (Slot &s : slots) {
        // slots belong to the scheduler thread: their events are queried and
        // their results copied out without holding the lock, so submitters
        // are never held up by a large group's copies
        if (!s.busy)
            continue;
        const int64_t q0 = now_ns();
        const hipError_t q = hipEventQuery(s.done);
        const int64_t seen = now_ns();
        step_query_ns = std::max(step_query_ns, seen - q0);
        st.max_query_ms = std::max(st.max_query_ms, static_cast<double>(seen - q0) * 1e-6);
        if (q != hipSuccess)
            continue;
        lk.unlock();
        copy_items.clear();
        for (Request *r : s.reqs) {
            const int64_t n = code_n[r->code_id];
            const int64_t e = s.elem_begin + r->elem_off;
            copy_items.push_back({r->bits, h_bits + e, static_cast<size_t>(r->frames * n)});
            copy_items.push_back({r->iters, h_iters + s.frame_begin + r->frame_off, sizeof(int32_t) * r->frames});
            if (r->post)
                copy_items.push_back({r->post, h_post + e, sizeof(float) * static_cast<size_t>(r->frames * n)});
        }
        copies->run(copy_items);
        const int64_t t = now_ns();
        lk.lock();
        step_copy_ns = std::max(step_copy_ns, t - seen);
        st.max_copy_ms = std::max(st.max_copy_ms, static_cast<double>(t - seen) * 1e-6);
        for (Request *r : s.reqs) {
            r->seen_ns = seen;
            r->done_ns = t;
            r->state = kDone;
            const double lat = static_cast<double>(t - r->arrival_ns) * 1e-6;
            lat_ms.push_back(lat);
            if (lat > worst_ms) {
                worst_ms = lat;
                st.worst_submit_ms = static_cast<double>(r->submit_ns - r->arrival_ns) * 1e-6;
                st.worst_queue_ms = static_cast<double>(r->admit_ns - r->submit_ns) * 1e-6;
                st.worst_stage_ms = static_cast<double>(r->launch_ns - r->admit_ns) * 1e-6;
                st.worst_device_ms = static_cast<double>(r->seen_ns - r->launch_ns) * 1e-6;
                st.worst_copyout_ms = static_cast<double>(r->done_ns - r->seen_ns) * 1e-6;
            }
            st.completed += 1;
            st.frames_completed += r->frames;
            st.bits_completed += r->frames * code_n[r->code_id];
        }
        s.reqs.clear();
        elems.release(s.elem_begin, s.elem_len);
        frames.release(s.frame_begin, s.frame_len);
        s.busy = false;
        any = true;
    }
    if (any)
        cv_done.notify_all();
    return any;
}

bool ldpc_server_s::admit(std::unique_lock<std::mutex> &lk)
{
    bool any = false;
    for (Slot &s : slots) {
        if (s.busy || queue.empty())
            continue;
        // longest FIFO prefix within the group cap ...
        size_t k = 0;
        int64_t f = 0, e = 0;
        while (k < queue.size() && f + queue[k]->frames <= max_group_frames) {
            f += queue[k]->frames;
            e += static_cast<int64_t>(queue[k]->frames) * code_n[queue[k]->code_id];
            ++k;
        }
        // ... that the arena can hold right now
        int64_t eb = -1, fb = -1;
        while (k > 0) {
            eb = elems.alloc(align4(e));
            if (eb >= 0) {
                fb = frames.alloc(f);
                if (fb >= 0)
                    break;
                elems.release(eb, align4(e));
                eb = -1;
            }
            --k;
            f -= queue[k]->frames;
            e -= static_cast<int64_t>(queue[k]->frames) * code_n[queue[k]->code_id];
        }
        if (k == 0)
            break;  // the head of the queue waits for memory (first come, first served)
        s.reqs.assign(queue.begin(), queue.begin() + static_cast<long>(k));
        queue.erase(queue.begin(), queue.begin() + static_cast<long>(k));
        s.elem_begin = eb;
        s.elem_len = align4(e);
        s.frame_begin = fb;
        s.frame_len = f;
        s.want_post = false;
        const int64_t admitted = now_ns();
        for (Request *r : s.reqs) {
            r->state = kInFlight;  // from here on cancel() refuses these requests
            r->admit_ns = admitted;
        }
        // staging copies and launches run without the lock
        lk.unlock();
        // The group's requests are laid out in the arena by code (and by
        // iteration limit, flags and whether posteriors are wanted), FIFO
        // within each, so that neighbours decoded alike merge into one job:
        // a group of many small requests becomes a few jobs and fits one
        // fused launch.
        std::stable_sort(s.reqs.begin(), s.reqs.end(), [](const Request *a, const Request *b) {
            if (a->code_id != b->code_id)
                return a->code_id < b->code_id;
            if (a->max_iter != b->max_iter)
                return a->max_iter < b->max_iter;
            if (a->flags != b->flags)
                return a->flags < b->flags;
            return (a->post != nullptr) < (b->post != nullptr);
        });
        jobs.clear();
        copy_items.clear();
        int64_t eo = 0, fo = 0;
        const Request *prev = nullptr;
        for (Request *r : s.reqs) {
            const int64_t n = code_n[r->code_id];
            r->elem_off = eo;
            r->frame_off = fo;
            copy_items.push_back({h_llr + eb + eo, r->llr, sizeof(float) * static_cast<size_t>(r->frames * n)});
            if (prev && prev->code_id == r->code_id && prev->max_iter == r->max_iter && prev->flags == r->flags &&
                (prev->post != nullptr) == (r->post != nullptr)) {
                jobs.back().frames += r->frames;  // contiguous with the previous request's frames
            } else {
                ldpc_job j{};
                j.code = codes[r->code_id];
                j.frames = r->frames;
                j.max_iter = r->max_iter;
                j.flags = r->flags;
                j.llr = d_llr + eb + eo;
                j.bits = dh_bits + eb + eo;
                j.iters = dh_iters + fb + fo;
                j.posterior = r->post ? dh_post + eb + eo : nullptr;
                jobs.push_back(j);
            }
            s.want_post |= r->post != nullptr;
            prev = r;
            eo += r->frames * n;
            fo += r->frames;
        }
        copies->run(copy_items);
        const int64_t copied = now_ns();
        // The copy kernel moves the staged LLRs into the device arena (the
        // decode kernel reads them every iteration); the decode kernel writes
        // bits, iteration counts and posteriors straight into pinned host
        // memory (each once).  The runtime's copy calls are not used here:
        // they have been seen to block the calling thread for milliseconds.
        ldpc_status rc =
            ldpc::launch_link_copy16(d_llr + eb, dh_llr + eb, sizeof(float) * static_cast<size_t>(align4(e)),
                                     kLinkCopyBlocks, s.stream);
        if (rc == LDPC_OK)
            rc = ldpc_decode_batch(jobs.data(), static_cast<int32_t>(jobs.size()), LDPC_F32, s.ws, s.ws_bytes,
                                   s.stream);
        if (rc != LDPC_OK) {
            // the group could not be launched: its requests complete with iteration count -1
            (void)hipStreamSynchronize(s.stream);
            for (Request *r : s.reqs)
                std::fill(r->iters, r->iters + r->frames, -1);
            const int64_t t = now_ns();
            lk.lock();
            for (Request *r : s.reqs) {
                r->done_ns = t;
                r->state = kDone;
                st.failed += 1;
            }
            s.reqs.clear();
            elems.release(eb, align4(e));
            frames.release(fb, f);
            cv_done.notify_all();
            any = true;
            continue;
        }
        (void)hipEventRecord(s.done, s.stream);
        const int64_t launched = now_ns();
        for (Request *r : s.reqs)
            r->launch_ns = launched;
        lk.lock();
        step_copy_ns = std::max(step_copy_ns, copied - admitted);
        step_launch_ns = std::max(step_launch_ns, launched - copied);
        st.max_copy_ms = std::max(st.max_copy_ms, static_cast<double>(copied - admitted) * 1e-6);
        st.max_launch_ms = std::max(st.max_launch_ms, static_cast<double>(launched - copied) * 1e-6);
        s.busy = true;
        st.launches += 1;
        group_frames_sum += f;
        any = true;
    }
    return any;
}

void ldpc_server_s::schedule(std::unique_lock<std::mutex> &lk)
{
    const bool tracing = !trace_path.empty();
    int64_t slept = 0;
    bool waited_busy = false;  // the last wait was a 20 us poll (with groups in flight)
    for (;;) {
        const int64_t t0 = now_ns();
        int64_t c0 = 0;
        rusage u0{};
        if (tracing) {
            c0 = thread_cpu_ns();
            getrusage(RUSAGE_THREAD, &u0);
            step_copy_ns = step_launch_ns = step_query_ns = 0;
        }
        reap(lk);
        admit(lk);
        const int64_t t1 = now_ns();
        st.max_step_ms = std::max(st.max_step_ms, static_cast<double>(t1 - t0) * 1e-6);
        if (tracing && (t1 - t0 > kTraceStepNs || (waited_busy && slept > kTraceStepNs))) {
            rusage u1{};
            getrusage(RUSAGE_THREAD, &u1);
            trace.push_back(StepTrace{t0 - t_created, t1 - t0, thread_cpu_ns() - c0, slept, step_copy_ns,
                                      step_launch_ns, step_query_ns, u1.ru_nvcsw - u0.ru_nvcsw,
                                      u1.ru_nivcsw - u0.ru_nivcsw});
        }
        const bool busy = std::any_of(slots.begin(), slots.end(), [](const Slot &s) { return s.busy; });
        if (stop && queue.empty() && !busy)
            break;
        waited_busy = busy;
        if (busy) {
            // Groups in flight: poll again within 20 us, or sooner once a
            // request arrives.  The thread spins rather than sleeps: waking a
            // sleeping thread has been seen to take milliseconds here, which
            // every request in flight would wait out.
            const uint64_t seen = submits.load(std::memory_order_relaxed);
            lk.unlock();
            const int64_t until = t1 + 20000;
            while (submits.load(std::memory_order_relaxed) == seen && now_ns() < until)
                __builtin_ia32_pause();
            lk.lock();
        } else {
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        }
        slept = now_ns() - t1;
    }
}

// A request completes as failed: every iteration count -1 (under the lock).
// One that already completed keeps its results.
void ldpc_server_s::fail_request(Request *r, int64_t t)
{
    if (r->state == kDone)
        return;
    std::fill(r->iters, r->iters + r->frames, -1);
    r->done_ns = t;
    r->state = kDone;
    st.failed += 1;
}

// After an exception in the scheduler (a host allocation failure): let every
// admitted group finish on the device, fail its requests and every queued
// one, and keep failing new ones until the server is destroyed.  Nothing
// here allocates.
void ldpc_server_s::fail_everything(std::unique_lock<std::mutex> &lk)
{
    if (!lk.owns_lock())
        lk.lock();
    broken = true;
    for (Slot &s : slots) {
        if (s.reqs.empty() && !s.busy)
            continue;
        lk.unlock();
        (void)hipStreamSynchronize(s.stream);
        lk.lock();
        const int64_t t = now_ns();
        for (Request *r : s.reqs)
            fail_request(r, t);
        s.reqs.clear();
        s.busy = false;
    }
    for (;;) {
        const int64_t t = now_ns();
        for (Request *r : queue)
            fail_request(r, t);
        queue.clear();
        cv_done.notify_all();
        if (stop)
            return;
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    }
}

void ldpc_server_s::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu, std::defer_lock);
    try {
        lk.lock();
        schedule(lk);
    } catch (...) {
        fail_everything(lk);
    }
}

void ldpc_server_s::free_all()
{
    for (Slot &s : slots) {
        if (s.stream)
            (void)hipStreamSynchronize(s.stream);
        if (s.done)
            (void)hipEventDestroy(s.done);
        if (s.stream)
            (void)hipStreamDestroy(s.stream);
        if (s.ws)
            (void)hipFree(s.ws);
    }
    if (d_llr)
        (void)hipFree(d_llr);
    if (h_llr)
        (void)hipHostFree(h_llr);
    for (Request *r : by_ticket)
        delete r;
    by_ticket.clear();
}

using namespace ldpc;

namespace {
// Releases a server that was never handed out (no scheduler thread yet).
struct ServerRelease {
    void operator()(ldpc_server_s *s) const
    {
        s->free_all();
        delete s;
    }
};
}  // namespace

extern "C" ldpc_status ldpc_server_create(const ldpc_server_cfg *cfg, ldpc_server *out)
try {
    if (!cfg || !out || cfg->ncodes < 1 || cfg->ncodes > 64 || !cfg->codes || cfg->max_inflight < 1 ||
        cfg->max_inflight > 8 || cfg->max_group_frames < 1 || cfg->max_queue < 1 || cfg->mem_budget_bytes == 0)
        return LDPC_EINVAL;
    // owned here until it is handed out: every early return (and any
    // exception) releases whatever was set up so far
    std::unique_ptr<ldpc_server_s, ServerRelease> sv(new ldpc_server_s());
    if (hipGetDevice(&sv->device) != hipSuccess)
        return LDPC_EDEVICE;
    int32_t nmin = INT32_MAX;
    for (int32_t i = 0; i < cfg->ncodes; ++i) {
        ldpc_code c = cfg->codes[i];
        if (!c || !code_on_current_device(c))
            return LDPC_EINVAL;
        if (ldpc_batch_fits_fused(c, LDPC_F32, nullptr) != LDPC_OK)
            return LDPC_EUNSUPPORTED;
        sv->codes.push_back(c);
        sv->code_n.push_back(c->n);
        nmin = std::min(nmin, c->n);
    }
    sv->max_group_frames = cfg->max_group_frames;
    sv->max_queue = cfg->max_queue;
    // Budget per element: 4 bytes of device LLR + 9 of pinned host memory
    // (staged LLR, bit, posterior), rounded as 10; per frame 4 (iteration count).
    const int64_t elems_cap = static_cast<int64_t>(cfg->mem_budget_bytes / 10) & ~int64_t(3);
    const int64_t frames_cap = elems_cap / nmin + 1;
    const size_t llr_bytes = align_up(static_cast<size_t>(elems_cap) * 4, 256);
    const size_t host_bytes = 2 * llr_bytes + align_up(static_cast<size_t>(frames_cap) * 4, 256) +
                              static_cast<size_t>(elems_cap);
    void *d = nullptr, *h = nullptr, *dh = nullptr;
    if (elems_cap < 4)
        return LDPC_EINVAL;
    if (hipMalloc(&d, llr_bytes) != hipSuccess)
        return LDPC_ENOMEM;
    sv->d_llr = static_cast<float *>(d);
    if (hipHostMalloc(&h, host_bytes, hipHostMallocDefault) != hipSuccess)
        return LDPC_ENOMEM;
    sv->h_llr = static_cast<float *>(h);  // owns the pinned block (freed through it)
    if (hipHostGetDevicePointer(&dh, h, 0) != hipSuccess)
        return LDPC_EDEVICE;
    auto carve = [&](void *base, float *&llr, float *&post, int32_t *&it, uint8_t *&bits) {
        char *p = static_cast<char *>(base);
        llr = reinterpret_cast<float *>(p);
        post = reinterpret_cast<float *>(p + llr_bytes);
        it = reinterpret_cast<int32_t *>(p + 2 * llr_bytes);
        bits = reinterpret_cast<uint8_t *>(p + 2 * llr_bytes + align_up(static_cast<size_t>(frames_cap) * 4, 256));
    };
    carve(h, sv->h_llr, sv->h_post, sv->h_iters, sv->h_bits);
    carve(dh, sv->dh_llr, sv->dh_post, sv->dh_iters, sv->dh_bits);
    sv->elems = RangeAlloc(elems_cap);
    sv->frames = RangeAlloc(frames_cap);
    sv->slots.resize(cfg->max_inflight);
    // A group's requests become at most one job each (alike neighbours
    // merge), and its jobs at most one fused launch each (codes that do not
    // fit one launch's LDS together split it), so max_group_frames launch
    // tables always suffice, whatever the mix of codes, iteration limits
    // and flags.
    const size_t ws_bytes = static_cast<size_t>(cfg->max_group_frames) * ldpc::fused_group_bytes();
    for (Slot &s : sv->slots) {
        s.ws_bytes = ws_bytes;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&s.ws, ws_bytes) != hipSuccess)
            return LDPC_ENOMEM;
    }
    // Warm-up: on every slot's stream, the staging copy at a small and a large
    // size, then one frame of every code for one iteration.  The runtime sets
    // up the hardware queue behind a stream and loads kernel variants on first
    // use, which takes milliseconds each time; paying for it here keeps it out
    // of the first requests' latency.  A code's degree bucket is the largest
    // one any group holding it can need, so these launches touch every kernel
    // variant later groups use.
    const size_t big = std::min<size_t>(static_cast<size_t>(elems_cap) * sizeof(float), size_t(4) << 20);
    std::memset(sv->h_llr, 0, big);  // the copies below leave zero LLRs for the warm-up decodes
    for (Slot &s : sv->slots) {
        for (const size_t len : {std::min<size_t>(big, 4096), big})
            if (launch_link_copy16(sv->d_llr, sv->dh_llr, len, kLinkCopyBlocks, s.stream) != LDPC_OK)
                return LDPC_EDEVICE;
        for (size_t i = 0; i < sv->codes.size(); ++i) {
            if (sv->code_n[i] > std::min<int64_t>(elems_cap, 1 << 16))
                continue;  // requests for such a code are refused at submit anyway
            ldpc_job j{};
            j.code = sv->codes[i];
            j.frames = 1;
            j.max_iter = 1;
            j.llr = sv->d_llr;
            j.bits = sv->dh_bits;
            j.iters = sv->dh_iters;
            const ldpc_status rc = ldpc_decode_batch(&j, 1, LDPC_F32, s.ws, s.ws_bytes, s.stream);
            if (rc != LDPC_OK)
                return rc;
        }
        if (hipStreamSynchronize(s.stream) != hipSuccess)
            return LDPC_EDEVICE;
    }
    const unsigned hw = std::thread::hardware_concurrency();
    sv->copies.reset(new CopyPool(static_cast<int>(std::min(3u, hw > 4 ? hw / 4 : 0u))));
    if (const char *tp = std::getenv("LDPC_SERVER_TRACE")) {
        sv->trace_path = tp;
        sv->trace.reserve(4096);
    }
    sv->t_created = now_ns();
    ldpc_server_s *raw = sv.get();
    sv->sched = std::thread([raw] { raw->run(); });
    *out = sv.release();
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_server_submit(ldpc_server sv, int32_t code_id, int32_t frames, int32_t max_iter,
                                          uint32_t flags, const float *llr, uint8_t *bits, int32_t *iters,
                                          float *posterior, int64_t arrival_ns, uint64_t *ticket)
try {
    if (!sv || !ticket || code_id < 0 || code_id >= static_cast<int32_t>(sv->codes.size()) || frames < 1 ||
        max_iter < 0 || (flags & ~LDPC_EARLY_STOP) != 0 || !llr || !bits || !iters)
        return LDPC_EINVAL;
    const int64_t need = static_cast<int64_t>(frames) * sv->code_n[code_id];
    if (frames > sv->max_group_frames || align4(need) > sv->elems.capacity())
        return LDPC_EINVAL;
    std::unique_ptr<Request> owned(new Request());
    Request *r = owned.get();
    r->code_id = code_id;
    r->frames = frames;
    r->max_iter = max_iter;
    r->flags = flags;
    r->llr = llr;
    r->bits = bits;
    r->iters = iters;
    r->post = posterior;
    r->submit_ns = now_ns();
    r->arrival_ns = arrival_ns > 0 ? arrival_ns : r->submit_ns;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->broken)
            return LDPC_ENOMEM;
        if (sv->stop || static_cast<int32_t>(sv->queue.size()) >= sv->max_queue)
            return LDPC_EBUSY;
        // insert into the ticket map, then the queue; undo the first if the second throws
        sv->by_ticket.push_back(r);  // at index next_ticket - 1
        try {
            sv->queue.push_back(r);
        } catch (...) {
            sv->by_ticket.pop_back();
            throw;
        }
        owned.release();  // owned by the server from here on
        r->ticket = sv->next_ticket++;
        sv->st.submitted += 1;
        sv->st.max_queue_depth = std::max<int64_t>(sv->st.max_queue_depth, static_cast<int64_t>(sv->queue.size()));
        *ticket = r->ticket;
    }
    sv->submits.fetch_add(1, std::memory_order_relaxed);
    sv->cv_work.notify_one();
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_server_poll(ldpc_server sv, uint64_t ticket, int32_t *done)
try {
    if (!sv || !done)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    Request *const found = sv->find_ticket(ticket);
    if (!found)
        return LDPC_EINVAL;
    const int s = found->state;
    *done = (s == kDone || s == kCancelled) ? 1 : 0;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_server_wait(ldpc_server sv, uint64_t ticket, double timeout_ms)
try {
    if (!sv)
        return LDPC_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    Request *const found = sv->find_ticket(ticket);
    if (!found)
        return LDPC_EINVAL;
    Request *r = found;
    const bool ok = sv->cv_done.wait_for(lk, std::chrono::microseconds(static_cast<int64_t>(timeout_ms * 1e3)),
                                         [&] { return r->state == kDone || r->state == kCancelled; });
    return ok ? LDPC_OK : LDPC_EBUSY;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_server_cancel(ldpc_server sv, uint64_t ticket)
try {
    if (!sv)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    Request *const found = sv->find_ticket(ticket);
    if (!found)
        return LDPC_EINVAL;
    Request *r = found;
    if (r->state != kQueued)
        return LDPC_EBUSY;
    sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), r));
    r->state = kCancelled;
    sv->st.cancelled += 1;
    sv->cv_done.notify_all();
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_server_stats_get(ldpc_server sv, ldpc_server_stats *out, int reset)
try {
    if (!sv || !out)
        return LDPC_EINVAL;
    // Only the snapshot is taken under the lock (a swap when resetting): the
    // percentiles are computed afterwards, so submitters and the scheduler
    // are not held up for the O(n) work.
    ldpc_server_stats s;
    std::deque<double> v;
    int64_t group_frames = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        s = sv->st;
        group_frames = sv->group_frames_sum;
        if (reset) {
            v.swap(sv->lat_ms);
            sv->st = ldpc_server_stats{};
            sv->group_frames_sum = 0;
            sv->worst_ms = -1.0;
        } else {
            v = sv->lat_ms;
        }
    }
    auto pct = [&](double q) {
        if (v.empty())
            return 0.0;
        const size_t k = std::min(v.size() - 1, static_cast<size_t>(q * static_cast<double>(v.size())));
        std::nth_element(v.begin(), v.begin() + static_cast<long>(k), v.end());
        return v[k];
    };
    s.p50_ms = pct(0.50);
    s.p99_ms = pct(0.99);
    s.p999_ms = pct(0.999);
    s.max_ms = v.empty() ? 0.0 : *std::max_element(v.begin(), v.end());
    s.mean_group_frames = s.launches ? static_cast<double>(group_frames) / static_cast<double>(s.launches) : 0.0;
    *out = s;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" void ldpc_server_destroy(ldpc_server sv)
try {
    if (!sv)
        return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->sched.joinable())
        sv->sched.join();
    if (!sv->trace_path.empty()) {
        if (FILE *f = std::fopen(sv->trace_path.c_str(), "a")) {
            std::fprintf(f, "# start_ms wall_ms cpu_ms sleep_before_ms copy_ms launch_ms query_ms nvcsw nivcsw\n");
            for (const StepTrace &t : sv->trace)
                std::fprintf(f, "%.3f %.3f %.3f %.3f %.3f %.3f %.3f %ld %ld\n", t.start_ns * 1e-6, t.wall_ns * 1e-6,
                             t.cpu_ns * 1e-6, t.sleep_ns * 1e-6, t.copy_ns * 1e-6, t.launch_ns * 1e-6,
                             t.query_ns * 1e-6, t.nvcsw, t.nivcsw);
            std::fclose(f);
        }
    }
    sv->free_all();
    delete sv;
} catch (...) {
}
