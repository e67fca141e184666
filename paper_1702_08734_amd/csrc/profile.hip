// Kernel timing with HIP events (mk_profile_enable / mk_profile_read).
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace mk {

namespace {
std::atomic<bool> g_enabled{false};
std::mutex g_mu;
std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_records;

void clear_locked() {
    for (auto& kv : g_records)
        for (auto& ev : kv.second) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    g_records.clear();
}
}  // namespace

bool profiling_enabled() { return g_enabled.load(std::memory_order_relaxed); }

ProfScope::ProfScope(const char* name, hipStream_t stream) : name_(name), stream_(stream) {
    if (!profiling_enabled()) return;
    if (hipEventCreate(&start_) != hipSuccess) {
        start_ = nullptr;
        return;
    }
    (void)hipEventRecord(start_, stream_);
}

ProfScope::~ProfScope() {
    if (!start_) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess) {
        (void)hipEventDestroy(start_);
        return;
    }
    (void)hipEventRecord(stop, stream_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_records[name_].emplace_back(start_, stop);
}

}  // namespace mk

extern "C" mk_status mk_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(mk::g_mu);
    if (on) mk::clear_locked();
    mk::g_enabled.store(on != 0);
    return MK_OK;
}

extern "C" mk_status mk_profile_read(const char* name, double* total_ms, int64_t* launches) {
    MK_REQUIRE(name && total_ms && launches, MK_ERR_INVALID_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(mk::g_mu);
    *total_ms = 0.0;
    *launches = 0;
    auto it = mk::g_records.find(name);
    if (it == mk::g_records.end()) return MK_OK;
    for (auto& ev : it->second) {
        MK_HIP(hipEventSynchronize(ev.second));
        float ms = 0.f;
        MK_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
        *total_ms += ms;
        *launches += 1;
    }
    return MK_OK;
}
