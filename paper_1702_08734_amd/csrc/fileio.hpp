// Binary files of resident objects (index, network): a fixed 8-byte magic, a
// format version, then raw little-endian arrays in a documented order.
// Device arrays go through one host staging copy per array.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"

namespace mk {

struct BinFile {
    FILE* f = nullptr;
    std::string path;
    BinFile(const char* p, const char* mode) : f(std::fopen(p, mode)), path(p) {}
    ~BinFile() {
        if (f) std::fclose(f);
    }
    BinFile(const BinFile&) = delete;
    BinFile& operator=(const BinFile&) = delete;
    bool ok() const { return f != nullptr; }
    bool put(const void* p, size_t n) { return n == 0 || std::fwrite(p, 1, n, f) == n; }
    bool get(void* p, size_t n) { return n == 0 || std::fread(p, 1, n, f) == n; }
    template <class T>
    bool put_v(const T& v) { return put(&v, sizeof(T)); }
    template <class T>
    bool get_v(T& v) { return get(&v, sizeof(T)); }
    // true when the whole file has been consumed
    bool at_end() { return std::fgetc(f) == EOF; }
    // close and report write errors that fclose flushes out
    bool close() {
        const bool good = std::fclose(f) == 0;
        f = nullptr;
        return good;
    }
};

// Copy `bytes` of device memory to the file through a host buffer.
inline mk_status put_device(BinFile& out, const void* dev, size_t bytes) {
    if (bytes == 0) return MK_OK;
    std::vector<unsigned char> h(bytes);
    MK_HIP(hipMemcpy(h.data(), dev, bytes, hipMemcpyDeviceToHost));
    MK_REQUIRE(out.put(h.data(), bytes), MK_ERR_INVALID_ARG, "write to " + out.path + " failed");
    return MK_OK;
}

// Read `bytes` from the file into device memory through a host buffer.
inline mk_status get_device(BinFile& in, void* dev, size_t bytes) {
    if (bytes == 0) return MK_OK;
    std::vector<unsigned char> h(bytes);
    MK_REQUIRE(in.get(h.data(), bytes), MK_ERR_INVALID_ARG, in.path + " is truncated");
    MK_HIP(hipMemcpy(dev, h.data(), bytes, hipMemcpyHostToDevice));
    return MK_OK;
}

}  // namespace mk
