// Library-wide C ABI helpers: version, the per-thread error message, the
// setting of the stream-ordered allocator's pool and the per-thread default
// scratch arena.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace mk {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }

// The default memory pool of each device keeps what the library's scratch
// allocations freed (release threshold: unlimited) instead of returning it
// at every synchronisation: a search allocates hundreds of MB of candidate
// pools and partial lists, and getting them afresh on each call slowed
// calls unevenly (k-selection of 10^4 rows of 1.28 10^5 at k = 1000:
// 1.50-1.81 ms over 20 calls, 1.44-1.55 ms with the memory kept; exact
// search at k = 1024: 37.0-37.7 ms, 36.8-37.0 ms kept).  The memory stays
// reserved for the process, up to the most the library held at once.
void keep_pool_memory() {
    static std::mutex mu;
    static std::vector<char> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)done.size() <= dev) done.resize(dev + 1, 0);
    if (done[dev]) return;
    done[dev] = 1;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess || !pool) return;
    uint64_t threshold = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
}

static thread_local Arena* g_thread_arena = nullptr;

Arena* thread_arena() { return g_thread_arena; }

ArenaScope::ArenaScope(Arena* a) : prev_(g_thread_arena) { g_thread_arena = a; }

ArenaScope::~ArenaScope() { g_thread_arena = prev_; }

}  // namespace mk

extern "C" const char* mk_last_error(void) { return mk::get_error(); }

extern "C" int32_t mk_version(void) { return 100; }
