// Shared host-side plumbing of the C ABI: status codes, the per-thread error
// message, HIP error checks and stream-ordered scratch allocations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "mi_knn.h"

namespace mk {

void set_error(const std::string& msg);
const char* get_error();
// Once per device: the default memory pool keeps freed scratch memory.
void keep_pool_memory();

#define MK_REQUIRE(cond, status, msg)                      \
    do {                                                   \
        if (!(cond)) {                                     \
            ::mk::set_error(std::string(__func__) + ": " + (msg)); \
            return (status);                               \
        }                                                  \
    } while (0)

#define MK_HIP(expr)                                                                 \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::mk::set_error(std::string(__func__) + ": " #expr " failed: " +         \
                            hipGetErrorString(e_));                                  \
            return e_ == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_DEVICE;           \
        }                                                                            \
    } while (0)

#define MK_LAUNCHED()                                                                \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess) {                                                      \
            ::mk::set_error(std::string(__func__) + ": kernel launch failed: " +     \
                            hipGetErrorString(e_));                                  \
            return MK_ERR_DEVICE;                                                    \
        }                                                                            \
    } while (0)

#define MK_TRY(expr)                  \
    do {                              \
        mk_status st_ = (expr);       \
        if (st_ != MK_OK) return st_; \
    } while (0)

// A caller-provided block of device memory that scratch buffers are carved
// from in order (256-byte aligned) instead of being allocated.  A sizing
// arena (sizing = true) hands out null pointers and only adds up the bytes a
// call would carve; code that receives one returns before launching work.
struct Arena {
    unsigned char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    bool sizing = false;
};

inline bool sizing_only(const Arena* a) { return a && a->sizing; }

// The calling thread's default arena: scratch requested without an explicit
// arena is carved from it while an ArenaScope is alive on that thread, and
// taken from the stream-ordered allocator when it does not fit (or when no
// scope is active).  A long-lived caller that launches one call at a time per
// stream (the serving loop: one workspace per stream) thereby makes no
// allocator calls per search.
Arena* thread_arena();
class ArenaScope {
public:
    explicit ArenaScope(Arena* a);
    ~ArenaScope();
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;

private:
    Arena* prev_;
};

// Device scratch: stream-ordered allocations freed on the same stream when
// they go out of scope (so a call never synchronises to release them), or,
// with an arena (explicit, else the thread's), a slice of the arena that is
// never freed.
struct Scratch {
    void* ptr = nullptr;
    hipStream_t stream = nullptr;
    bool owned = false;
    Scratch() = default;
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    mk_status alloc(size_t bytes, hipStream_t s, Arena* arena = nullptr) {
        stream = s;
        if (bytes == 0) bytes = 256;
        if (arena) {
            const size_t start = (arena->used + 255) & ~(size_t)255;
            if (arena->sizing) {
                ptr = nullptr;
                arena->used = start + bytes;
                owned = false;
                return MK_OK;
            }
            if (start > arena->size || bytes > arena->size - start) {
                set_error("scratch of " + std::to_string(bytes) + " bytes does not fit the " +
                          std::to_string(arena->size) + "-byte workspace (" +
                          std::to_string(start) + " bytes already used)");
                return MK_ERR_UNSUPPORTED;
            }
            ptr = arena->base + start;
            arena->used = start + bytes;
            owned = false;
            return MK_OK;
        }
        if (Arena* t = thread_arena()) {
            const size_t start = (t->used + 255) & ~(size_t)255;
            if (start <= t->size && bytes <= t->size - start) {
                ptr = t->base + start;
                t->used = start + bytes;
                owned = false;
                return MK_OK;
            }
        }
        keep_pool_memory();
        hipError_t e = hipMallocAsync(&ptr, bytes, s);
        if (e != hipSuccess) {
            ptr = nullptr;
            set_error(std::string("scratch allocation of ") + std::to_string(bytes) +
                      " bytes failed: " + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_DEVICE;
        }
        owned = true;
        return MK_OK;
    }
    template <class T>
    T* as() const { return static_cast<T*>(ptr); }
    ~Scratch() {
        if (ptr && owned) (void)hipFreeAsync(ptr, stream);
    }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mk
