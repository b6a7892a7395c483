// Per-kernel device timing with HIP events carried by the launches themselves
// (measurement aid, off by default).
#include <atomic>
#include <mutex>
#include <vector>

#include "ldpc_internal.h"

namespace {

struct Record {
    int kind;
    hipEvent_t start, stop;
};

std::atomic<int> g_enabled{0};
std::mutex g_mu;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event()
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_pool.empty()) {
            hipEvent_t e = g_pool.back();
            g_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

}  // namespace

ldpc::ProfScope::ProfScope(ldpc_kernel_kind kind, hipStream_t stream, bool enabled)
{
    if (!enabled || !g_enabled.load(std::memory_order_relaxed) || capturing(stream))
        return;
    start_ = take_event();
    stop_ = start_ ? take_event() : nullptr;
    if (!stop_) {
        if (start_) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_pool.push_back(start_);
        }
        start_ = nullptr;
        return;
    }
    kind_ = kind;
}

ldpc::ProfScope::~ProfScope()
{
    if (!start_)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_records.push_back({kind_, start_, stop_});
}

extern "C" ldpc_status ldpc_profile_enable(int enable)
try {
    g_enabled.store(enable ? 1 : 0);
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_profile_collect(double *ms, int64_t *counts)
try {
    std::vector<Record> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        recs.swap(g_records);
    }
    double acc[LDPC_KERNEL_KINDS] = {0};
    int64_t cnt[LDPC_KERNEL_KINDS] = {0};
    ldpc_status st = LDPC_OK;
    for (const Record &r : recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess)
            st = LDPC_EDEVICE;
        acc[r.kind] += t;
        cnt[r.kind] += 1;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Record &r : recs) {
            g_pool.push_back(r.start);
            g_pool.push_back(r.stop);
        }
    }
    for (int k = 0; k < LDPC_KERNEL_KINDS; ++k) {
        if (ms)
            ms[k] = acc[k];
        if (counts)
            counts[k] = cnt[k];
    }
    return st;
} catch (...) {
    return ldpc::status_of_exception();
}
