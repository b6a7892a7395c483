// The paper's multi-stream structure, as a measured baseline.
//
// Section III-C: W host worker threads, each controlling its own GPU stream
// and its own set of F frames; a worker interleaves, decodes and
// de-interleaves its frames (kernels 1, 2, 3 of Section III-B) on its stream,
// so W x F frames are in flight.  Here each worker repeatedly takes the next
// batch of F frames from a shared counter, copies its LLRs into pinned host
// staging and to the device, decodes them with ldpc_decode (whose ingest and
// output kernels are the interleaving kernels), copies bits and iteration
// counts back, waits for its stream and copies the results out.  The host
// cost of this structure (the workers' copies, launches and waits) is
// measured with getrusage over the run, next to the throughput.
#include <sys/resource.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <unistd.h>
#include <vector>

#include "ldpc_internal.h"

namespace {

double now_ms()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return static_cast<double>(ts.tv_sec) * 1e3 + static_cast<double>(ts.tv_nsec) * 1e-6;
}

double cpu_ms()
{
    rusage ru{};
    getrusage(RUSAGE_SELF, &ru);
    return (static_cast<double>(ru.ru_utime.tv_sec + ru.ru_stime.tv_sec) * 1e3 +
            static_cast<double>(ru.ru_utime.tv_usec + ru.ru_stime.tv_usec) * 1e-3);
}

struct Worker {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float *h_llr = nullptr;
    uint8_t *h_bits = nullptr;
    int32_t *h_iters = nullptr;
    float *d_llr = nullptr;
    uint8_t *d_bits = nullptr;
    int32_t *d_iters = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;

    void release()
    {
        if (stream)
            (void)hipStreamSynchronize(stream);
        if (done)
            (void)hipEventDestroy(done);
        if (stream)
            (void)hipStreamDestroy(stream);
        for (void *p : {static_cast<void *>(h_llr), static_cast<void *>(h_bits), static_cast<void *>(h_iters)})
            if (p)
                (void)hipHostFree(p);
        for (void *p : {static_cast<void *>(d_llr), static_cast<void *>(d_bits), static_cast<void *>(d_iters), ws})
            if (p)
                (void)hipFree(p);
    }
};

}  // namespace

extern "C" ldpc_status ldpc_mstream_run(ldpc_code code, int32_t workers, int32_t frames_per_batch, int32_t batches,
                                        int32_t max_iter, uint32_t flags, int32_t blocking_sync, const float *llr,
                                        uint8_t *bits, int32_t *iters, ldpc_mstream_stats *stats)
try {
    if (!code || workers < 1 || workers > 64 || frames_per_batch < 1 || frames_per_batch > LDPC_MAX_FRAMES ||
        batches < 0 || max_iter < 0 || (flags & ~(LDPC_EARLY_STOP | LDPC_LAYERED | LDPC_MIN_SUM)) != 0 ||
        (batches > 0 && (!llr || !bits || !iters)))
        return LDPC_EINVAL;
    if (!ldpc::code_on_current_device(code))
        return LDPC_EINVAL;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return LDPC_EDEVICE;
    const int64_t n = code->n;
    const int64_t F = frames_per_batch;
    const size_t llr_bytes = static_cast<size_t>(F * n) * sizeof(float);
    const size_t ws_bytes = ldpc::stream_workspace_bytes(code, LDPC_F32, frames_per_batch, max_iter);

    std::vector<Worker> ws(static_cast<size_t>(workers));
    ldpc_status st = LDPC_OK;
    for (Worker &w : ws) {
        w.ws_bytes = ws_bytes;
        if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&w.done, blocking_sync ? (hipEventBlockingSync | hipEventDisableTiming)
                                                           : hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&w.h_llr), llr_bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&w.h_bits), static_cast<size_t>(F * n), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&w.h_iters), static_cast<size_t>(F) * sizeof(int32_t),
                          hipHostMallocDefault) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&w.d_llr), llr_bytes) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&w.d_bits), static_cast<size_t>(F * n)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&w.d_iters), static_cast<size_t>(F) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&w.ws, ws_bytes) != hipSuccess) {
            st = LDPC_ENOMEM;
            break;
        }
    }
    if (st != LDPC_OK) {
        for (Worker &w : ws)
            w.release();
        return st;
    }

    std::atomic<int32_t> next{0};
    std::atomic<int> failed{LDPC_OK};
    auto work = [&](Worker &w) {
        (void)hipSetDevice(device);
        for (;;) {
            const int32_t b = next.fetch_add(1);
            if (b >= batches || failed.load() != LDPC_OK)
                return;
            const size_t base = static_cast<size_t>(b) * static_cast<size_t>(F * n);
            std::memcpy(w.h_llr, llr + base, llr_bytes);
            ldpc_status rc = LDPC_OK;
            if (hipMemcpyAsync(w.d_llr, w.h_llr, llr_bytes, hipMemcpyHostToDevice, w.stream) != hipSuccess)
                rc = LDPC_EDEVICE;
            if (rc == LDPC_OK)
                rc = ldpc_decode(code, LDPC_F32, frames_per_batch, max_iter, flags, w.d_llr, w.d_bits, w.d_iters,
                                 nullptr, w.ws, w.ws_bytes, w.stream);
            if (rc == LDPC_OK &&
                (hipMemcpyAsync(w.h_bits, w.d_bits, static_cast<size_t>(F * n), hipMemcpyDeviceToHost, w.stream) !=
                     hipSuccess ||
                 hipMemcpyAsync(w.h_iters, w.d_iters, static_cast<size_t>(F) * sizeof(int32_t),
                                hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
                 hipEventRecord(w.done, w.stream) != hipSuccess || hipEventSynchronize(w.done) != hipSuccess))
                rc = LDPC_EDEVICE;
            if (rc != LDPC_OK) {
                int expected = LDPC_OK;
                failed.compare_exchange_strong(expected, static_cast<int>(rc));
                return;
            }
            std::memcpy(bits + base, w.h_bits, static_cast<size_t>(F * n));
            std::memcpy(iters + static_cast<size_t>(b) * static_cast<size_t>(F), w.h_iters,
                        static_cast<size_t>(F) * sizeof(int32_t));
        }
    };

    const double c0 = cpu_ms(), t0 = now_ms();
    std::vector<std::thread> threads;
    threads.reserve(ws.size());
    for (Worker &w : ws)
        threads.emplace_back(work, std::ref(w));
    for (std::thread &t : threads)
        t.join();
    const double t1 = now_ms(), c1 = cpu_ms();
    for (Worker &w : ws)
        w.release();
    if (failed.load() != LDPC_OK)
        return static_cast<ldpc_status>(failed.load());
    if (stats) {
        const double wall = t1 - t0;
        const long cores = std::max(1L, sysconf(_SC_NPROCESSORS_ONLN));
        stats->wall_ms = wall;
        stats->frames_per_s = wall > 0 ? static_cast<double>(batches) * F / (wall * 1e-3) : 0.0;
        stats->mbps = stats->frames_per_s * static_cast<double>(n) * 1e-6;
        stats->cpu_ms = c1 - c0;
        stats->cpu_cores_busy = wall > 0 ? (c1 - c0) / wall : 0.0;
        stats->cpu_load = stats->cpu_cores_busy / static_cast<double>(cores);
        stats->online_cores = static_cast<int32_t>(cores);
    }
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}
