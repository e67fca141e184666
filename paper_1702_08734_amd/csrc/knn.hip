// Exact k-NN search (Section 2 Eq. 1-2, Section 5.1).
//
// Layout of one call:
//   1. norms: ||y||^2 per database row (one pass, Eq. 2), skipped for inner
//      products or when the caller supplies them;
//   2. knn_fused (fused.hpp): the grid is (query block) x (database chunk).
//      Producer waves keep their queries' MFMA A-operands in registers,
//      stream the chunk in 64-row tiles into LDS with direct global-to-LDS
//      loads one tile ahead, compute the q.y tile with v_mfma_f32_16x16x4f32
//      and stage it in LDS; consumer waves turn it into scores
//      (||y||^2 - 2 q.y for L2, -q.y for inner products; ||x||^2 is constant
//      per query and not needed to rank, Section 5.1) and feed them to
//      register-resident selectors -- distance computation and k-selection in
//      one kernel, so the distance matrix never reaches HBM;
//   3. knn_merge_rerank: one wave per query selects the best of the chunks'
//      partial lists (the second pass of Section 5.3's two-pass selection),
//      recomputes the kept candidates' distances in the direct form in FP32,
//      and re-ranks them.  The selection keeps k + 16 candidates (when the
//      1024-entry queue allows) so that the FP32 cancellation of the norm
//      decomposition cannot push a true neighbour out of the final k.
#include <algorithm>
#include <mutex>
#include <vector>

#include "fused.hpp"

namespace mk {

// ---------------------------------------------------------------- norms
// One 16-lane group per row, so that a wave's loads are coalesced 16-byte
// granules of four rows at a time (one row per lane read each row as 64
// scattered streams: about 1 TB/s); the group's partial sums meet through
// lane shuffles.  Grid-stride over groups of four rows.
__global__ __launch_bounds__(256) void norms_kernel(const float* __restrict__ x, int64_t n,
                                                    int32_t d, float* __restrict__ out) {
    const int lane = threadIdx.x & 63, sub = lane >> 4, l16 = lane & 15;
    const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    for (int64_t r0 = w0 * 4; r0 < n; r0 += nw * 4) {
        const int64_t i = r0 + sub;
        float s = 0.f;
        if (i < n) {
            const float* p = x + i * d;
            if (vec) {
                for (int t = l16 * 4; t < d; t += 64) {
                    const float4 v = *reinterpret_cast<const float4*>(p + t);
                    s = fmaf(v.x, v.x, s);
                    s = fmaf(v.y, v.y, s);
                    s = fmaf(v.z, v.z, s);
                    s = fmaf(v.w, v.w, s);
                }
            } else {
                for (int t = l16; t < d; t += 16) s = fmaf(p[t], p[t], s);
            }
        }
        s += __shfl_xor(s, 8, 16);
        s += __shfl_xor(s, 4, 16);
        s += __shfl_xor(s, 2, 16);
        s += __shfl_xor(s, 1, 16);
        if (l16 == 0 && i < n) out[i] = s;
    }
}

mk_status launch_norms(const float* x, int64_t n, int32_t d, float* out, hipStream_t s) {
    if (n == 0) return MK_OK;
    const int64_t blocks = ceil_div(n, 16);  // four rows per wave, four waves per block
    hipLaunchKernelGGL(norms_kernel, dim3((unsigned)(blocks < 32768 ? blocks : 32768)), dim3(256), 0,
                       s, x, n, d, out);
    MK_LAUNCHED();
    return MK_OK;
}


// Fused search for padded dimension class DP (knn_impl.hpp, one translation
// unit per class).
template <int DP>
mk_status knn_dispatch_k(const float* xq, int64_t nq, const float* xb, const float* yn,
                         int64_t nb, int32_t d, int32_t k, bool l2, bool vec, float* D, int64_t* I,
                         hipStream_t s, Arena* arena);
extern template mk_status knn_dispatch_k<32>(const float*, int64_t, const float*, const float*,
                                              int64_t, int32_t, int32_t, bool, bool, float*,
                                              int64_t*, hipStream_t, Arena*);
extern template mk_status knn_dispatch_k<64>(const float*, int64_t, const float*, const float*,
                                              int64_t, int32_t, int32_t, bool, bool, float*,
                                              int64_t*, hipStream_t, Arena*);
extern template mk_status knn_dispatch_k<96>(const float*, int64_t, const float*, const float*,
                                              int64_t, int32_t, int32_t, bool, bool, float*,
                                              int64_t*, hipStream_t, Arena*);
extern template mk_status knn_dispatch_k<128>(const float*, int64_t, const float*, const float*,
                                               int64_t, int32_t, int32_t, bool, bool, float*,
                                               int64_t*, hipStream_t, Arena*);
extern template mk_status knn_dispatch_k<256>(const float*, int64_t, const float*, const float*,
                                               int64_t, int32_t, int32_t, bool, bool, float*,
                                               int64_t*, hipStream_t, Arena*);

mk_status knn_search(const float* xq, int64_t nq, const float* xb, const float* yn_in, int64_t nb,
                     int32_t d, int32_t k, mk_metric metric, float* D, int64_t* I,
                     hipStream_t s, Arena* arena) {
    MK_REQUIRE(nq >= 0 && nb >= 0, MK_ERR_INVALID_ARG, "nq and nb must be >= 0");
    MK_REQUIRE(d >= 1, MK_ERR_INVALID_ARG, "d must be >= 1");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1024");
    MK_REQUIRE(d <= 256, MK_ERR_UNSUPPORTED, "d must be <= 256");
    MK_REQUIRE(nb < (1ll << 31), MK_ERR_UNSUPPORTED, "nb must be < 2^31");
    MK_REQUIRE(metric == MK_METRIC_L2 || metric == MK_METRIC_IP, MK_ERR_INVALID_ARG, "bad metric");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I && (xb || nb == 0), MK_ERR_INVALID_ARG, "null pointer");
    const bool l2 = metric == MK_METRIC_L2;
    const bool vec = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(xq) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(xb) % 16 == 0);
    Scratch norms;
    const float* yn = yn_in;
    if (l2 && !yn && nb > 0) {
        mk_status st = norms.alloc(sizeof(float) * (size_t)nb, s, arena);
        if (st != MK_OK) return st;
        if (!sizing_only(arena)) {
            st = launch_norms(xb, nb, d, norms.as<float>(), s);
            if (st != MK_OK) return st;
        }
        yn = norms.as<float>();
    }
    if (d <= 32) return knn_dispatch_k<32>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
    if (d <= 64) return knn_dispatch_k<64>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
    if (d <= 96) return knn_dispatch_k<96>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
    if (d <= 128) return knn_dispatch_k<128>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
    return knn_dispatch_k<256>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
}

// ------------------------------------------------- device symbols
// Count of candidates dropped by full candidate pools (debug; stays zero).
static __device__ unsigned long long pool_drops;

namespace {
std::mutex g_sym_mu;
std::vector<unsigned long long*> g_drops_dev;  // per device id; null until looked up
}  // namespace

mk_status pool_drop_counter(unsigned long long** out) {
    int dev = 0;
    MK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_sym_mu);
    if ((int)g_drops_dev.size() <= dev) g_drops_dev.resize(dev + 1, nullptr);
    if (!g_drops_dev[dev]) {
        void* p = nullptr;
        MK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(pool_drops)));
        MK_REQUIRE(p, MK_ERR_DEVICE, "no device address for the pool-drop counter");
        g_drops_dev[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_drops_dev[dev];
    return MK_OK;
}


// k-NN graph rows: the k + 1 best of node q minus the node itself (if it is
// among them), first k kept.  One thread per node.
__global__ void drop_node_kernel(const float* __restrict__ D1, const int64_t* __restrict__ I1,
                                 int64_t n, int32_t k, int64_t node0, float* __restrict__ D,
                                 int64_t* __restrict__ I) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int64_t self = node0 + q;
    const float* d1 = D1 + q * (k + 1);
    const int64_t* i1 = I1 + q * (k + 1);
    int32_t o = 0;
    for (int32_t j = 0; j <= k && o < k; ++j) {
        if (i1[j] == self) continue;
        D[q * k + o] = d1[j];
        I[q * k + o] = i1[j];
        ++o;
    }
}

// Chunk c's exact results (D, I local to the chunk) as merge keys in
// keys[q][c][k]: (distance, global row) for L2, (-product, global row) for
// inner products; padding entries (I = -1) become sentinels.
__global__ void chunk_keys_kernel(const float* __restrict__ D, const int64_t* __restrict__ I,
                                  int64_t nq, int32_t k, int32_t c, int32_t nchunks,
                                  int64_t row0, int32_t largest, uint64_t* __restrict__ keys) {
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < nq * k;
         g += (int64_t)gridDim.x * 256) {
        const int64_t q = g / k, j = g % k;
        const int64_t i = I[g];
        keys[(q * nchunks + c) * k + j] =
            i < 0 ? kSentinel : make_key(largest ? -D[g] : D[g], (uint32_t)(row0 + i));
    }
}

template <int KR>
mk_status rerank_launch(const uint64_t* keys, int64_t nq, int32_t R, const float* xq,
                        const float* xb, int32_t d, bool l2, bool vec, int32_t k, float* D,
                        int64_t* I, hipStream_t s) {
    ProfScope prof("rerank", s);
    // a workgroup per query: a quarter of the gather latency per query, and
    // a quarter of the LDS per workgroup of the wave-per-query merge kernel,
    // so more waves in flight (10^4 queries, R = 1024, 5*10^7 x 128 rows:
    // 0.99 ms against 1.44 ms; 64 queries: 0.06 against 0.22 ms)
    hipLaunchKernelGGL((knn_rerank_block<KR>), dim3((unsigned)nq), dim3(64 * kMergeWaves), 0, s,
                       keys, R, xq, xb, d, (int32_t)vec, (int32_t)l2, k, D, I);
    MK_LAUNCHED();
    return MK_OK;
}

mk_status rerank_keys(const uint64_t* keys, int64_t nq, int32_t R, const float* xq,
                      const float* xb, int32_t d, bool l2, int32_t k, float* D, int64_t* I,
                      hipStream_t s) {
    MK_REQUIRE(d >= 1 && d <= kMaxDim, MK_ERR_UNSUPPORTED, "re-rank needs 1 <= d <= 512");
    MK_REQUIRE(k >= 1 && k <= R && R <= kMaxK, MK_ERR_INVALID_ARG, "need 1 <= k <= R <= 1024");
    if (nq == 0) return MK_OK;
    const bool vec = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(xq) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(xb) % 16 == 0);
    switch (queue_regs(R)) {
        case 1: return rerank_launch<1>(keys, nq, R, xq, xb, d, l2, vec, k, D, I, s);
        case 2: return rerank_launch<2>(keys, nq, R, xq, xb, d, l2, vec, k, D, I, s);
        case 4: return rerank_launch<4>(keys, nq, R, xq, xb, d, l2, vec, k, D, I, s);
        case 8: return rerank_launch<8>(keys, nq, R, xq, xb, d, l2, vec, k, D, I, s);
        default: return rerank_launch<16>(keys, nq, R, xq, xb, d, l2, vec, k, D, I, s);
    }
}

}  // namespace mk

extern "C" mk_status mk_norms(const float* x, int64_t n, int32_t d, float* out,
                              mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1, MK_ERR_INVALID_ARG, "n must be >= 0 and d >= 1");
    if (n == 0) return MK_OK;
    MK_REQUIRE(x && out, MK_ERR_INVALID_ARG, "null pointer");
    return mk::launch_norms(x, n, d, out, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_knn_search(const float* xq, int64_t nq, const float* xb, int64_t nb,
                                   int32_t d, int32_t k, mk_metric metric, float* D, int64_t* I,
                                   mk_stream_t stream) {
    return mk::knn_search(xq, nq, xb, nullptr, nb, d, k, metric, D, I,
                          static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_knn_search_prenorm(const float* xq, int64_t nq, const float* xb,
                                           const float* yn, int64_t nb, int32_t d, int32_t k,
                                           mk_metric metric, float* D, int64_t* I,
                                           mk_stream_t stream) {
    MK_REQUIRE(metric != MK_METRIC_L2 || yn || nb == 0, MK_ERR_INVALID_ARG,
               "L2 search needs the database norms");
    return mk::knn_search(xq, nq, xb, yn, nb, d, k, metric, D, I,
                          static_cast<hipStream_t>(stream));
}

// ------------------------------------------------- allocation-free search
// The scratch of mk_knn_search_noalloc: database norms, chunk partial keys
// and rank points of one call, carved from a fixed array that every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is not a device address; only the address returned by
// hipGetSymbolAddress on the device in question is passed to kernels.
static __device__ __align__(256) unsigned char scratch[MK_NOALLOC_SCRATCH_BYTES];

namespace mk {
namespace {
std::vector<unsigned char*> g_scratch_dev;  // per device id; null until looked up
}  // namespace

mk_status noalloc_scratch(unsigned char** out) {
    int dev = 0;
    MK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_sym_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        MK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MK_REQUIRE(p, MK_ERR_DEVICE, "no device address for the search scratch array");
        g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return MK_OK;
}
}  // namespace mk

extern "C" mk_status mk_knn_search_noalloc(const float* xq, int64_t nq, const float* xb,
                                           int64_t nb, int32_t d, int32_t k, mk_metric metric,
                                           float* D, int64_t* I, mk_stream_t stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // Size the call first (validates the arguments, launches nothing).
    mk::Arena need;
    need.sizing = true;
    MK_TRY(mk::knn_search(xq, nq, xb, nullptr, nb, d, k, metric, D, I, s, &need));
    if (nq == 0) return MK_OK;
    MK_REQUIRE(need.used <= (size_t)MK_NOALLOC_SCRATCH_BYTES, MK_ERR_UNSUPPORTED,
               "the search needs " + std::to_string(need.used) +
                   " bytes of scratch, more than the " +
                   std::to_string((size_t)MK_NOALLOC_SCRATCH_BYTES) +
                   "-byte fixed array; split the queries into smaller batches");
    unsigned char* base = nullptr;
    MK_TRY(mk::noalloc_scratch(&base));
    mk::Arena arena;
    arena.base = base;
    arena.size = MK_NOALLOC_SCRATCH_BYTES;
    return mk::knn_search(xq, nq, xb, nullptr, nb, d, k, metric, D, I, s, &arena);
}

extern "C" mk_status mk_knn_graph(const float* xb, int64_t nb, int32_t d, int32_t k,
                                  mk_metric metric, int64_t node0, int64_t nnodes, float* D,
                                  int64_t* I, mk_stream_t stream) {
    MK_REQUIRE(nb >= 0 && node0 >= 0 && nnodes >= 0 && node0 + nnodes <= nb, MK_ERR_INVALID_ARG,
               "nodes node0 .. node0 + nnodes - 1 must be rows of xb");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k < mk::kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1023");
    if (nnodes == 0) return MK_OK;
    MK_REQUIRE(xb && D && I, MK_ERR_INVALID_ARG, "null pointer");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    mk::Scratch D1, I1;
    MK_TRY(D1.alloc(sizeof(float) * (size_t)nnodes * (k + 1), s));
    MK_TRY(I1.alloc(sizeof(int64_t) * (size_t)nnodes * (k + 1), s));
    MK_TRY(mk::knn_search(xb + node0 * d, nnodes, xb, nullptr, nb, d, k + 1, metric,
                          D1.as<float>(), I1.as<int64_t>(), s));
    hipLaunchKernelGGL(mk::drop_node_kernel, dim3((unsigned)mk::ceil_div(nnodes, 256)), dim3(256),
                       0, s, D1.as<float>(), I1.as<int64_t>(), nnodes, k, node0, D, I);
    MK_LAUNCHED();
    return MK_OK;
}

extern "C" mk_status mk_knn_search_host(const float* xq, int64_t nq, const float* xb_host,
                                        int64_t nb, int32_t d, int32_t k, mk_metric metric,
                                        int64_t chunk_rows, float* D, int64_t* I,
                                        mk_stream_t stream) {
    MK_REQUIRE(nq >= 0 && nb >= 0, MK_ERR_INVALID_ARG, "nq and nb must be >= 0");
    MK_REQUIRE(d >= 1 && d <= 256, MK_ERR_UNSUPPORTED, "d must be in [1, 256]");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= mk::kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1024");
    MK_REQUIRE(nb < 0xFFFFFFFFll, MK_ERR_UNSUPPORTED, "nb must be < 2^32 - 1");
    MK_REQUIRE(chunk_rows >= 1 && chunk_rows < (1ll << 31), MK_ERR_INVALID_ARG,
               "chunk_rows must be in [1, 2^31)");
    MK_REQUIRE(metric == MK_METRIC_L2 || metric == MK_METRIC_IP, MK_ERR_INVALID_ARG, "bad metric");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I && (xb_host || nb == 0), MK_ERR_INVALID_ARG, "null pointer");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool largest = metric == MK_METRIC_IP;
    if (nb <= chunk_rows) {
        // one chunk: copy and search in order on the caller's stream
        mk::Scratch buf;
        MK_TRY(buf.alloc(sizeof(float) * (size_t)(nb > 0 ? nb : 1) * d, s));
        if (nb > 0)
            MK_HIP(hipMemcpyAsync(buf.ptr, xb_host, sizeof(float) * (size_t)nb * d,
                                  hipMemcpyHostToDevice, s));
        MK_TRY(mk::knn_search(xq, nq, buf.as<float>(), nullptr, nb, d, k, metric, D, I, s));
        MK_HIP(hipStreamSynchronize(s));
        return MK_OK;
    }
    const int64_t nchunks = mk::ceil_div(nb, chunk_rows);
    MK_REQUIRE(nchunks <= (1 << 20), MK_ERR_INVALID_ARG, "too many chunks");
    mk::Scratch buf[2], Dc, Ic, keys;
    for (auto& b : buf) MK_TRY(b.alloc(sizeof(float) * (size_t)chunk_rows * d, s));
    MK_TRY(Dc.alloc(sizeof(float) * (size_t)nq * k, s));
    MK_TRY(Ic.alloc(sizeof(int64_t) * (size_t)nq * k, s));
    MK_TRY(keys.alloc(sizeof(uint64_t) * (size_t)nq * nchunks * k, s));
    // copies run on a second stream, one chunk ahead of the searches: the
    // copy of chunk c + 1 overlaps the search of chunk c; the copy into a
    // buffer waits for the search that last read it
    hipStream_t cs = nullptr;
    MK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr}, start = nullptr;
    mk_status st = MK_OK;
    auto fail = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && st == MK_OK) {
            mk::set_error(std::string("mk_knn_search_host: ") + what + ": " + hipGetErrorString(e));
            st = e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_DEVICE;
        }
        return st != MK_OK;
    };
    for (int i = 0; i < 2 && st == MK_OK; ++i) {
        fail(hipEventCreateWithFlags(&ready[i], hipEventDisableTiming), "event");
        fail(hipEventCreateWithFlags(&freed[i], hipEventDisableTiming), "event");
    }
    if (st == MK_OK) fail(hipEventCreateWithFlags(&start, hipEventDisableTiming), "event");
    // the staging buffers come from the caller's stream's allocator
    if (st == MK_OK) fail(hipEventRecord(start, s), "record");
    if (st == MK_OK) fail(hipStreamWaitEvent(cs, start, 0), "wait");
    auto copy = [&](int64_t c) {
        const int64_t r0 = c * chunk_rows;
        const int64_t n = nb - r0 < chunk_rows ? nb - r0 : chunk_rows;
        const int b = (int)(c & 1);
        if (c >= 2 && fail(hipStreamWaitEvent(cs, freed[b], 0), "wait")) return;
        if (fail(hipMemcpyAsync(buf[b].ptr, xb_host + r0 * d, sizeof(float) * (size_t)n * d,
                                hipMemcpyHostToDevice, cs), "copy"))
            return;
        fail(hipEventRecord(ready[b], cs), "record");
    };
    if (st == MK_OK) copy(0);
    for (int64_t c = 0; c < nchunks && st == MK_OK; ++c) {
        if (c + 1 < nchunks) copy(c + 1);
        if (st != MK_OK) break;
        const int b = (int)(c & 1);
        const int64_t r0 = c * chunk_rows;
        const int64_t n = nb - r0 < chunk_rows ? nb - r0 : chunk_rows;
        if (fail(hipStreamWaitEvent(s, ready[b], 0), "wait")) break;
        st = mk::knn_search(xq, nq, buf[b].as<float>(), nullptr, n, d, k, metric, Dc.as<float>(),
                            Ic.as<int64_t>(), s);
        if (st != MK_OK) break;
        hipLaunchKernelGGL(mk::chunk_keys_kernel,
                           dim3((unsigned)std::min<int64_t>(mk::ceil_div(nq * k, 256), 1 << 20)),
                           dim3(256), 0, s, Dc.as<float>(), Ic.as<int64_t>(), nq, k, (int32_t)c,
                           (int32_t)nchunks, r0, (int32_t)largest, keys.as<uint64_t>());
        if (fail(hipGetLastError(), "launch")) break;
        fail(hipEventRecord(freed[b], s), "record");
    }
    if (st == MK_OK)
        st = mk::merge_key_lists(keys.as<uint64_t>(), nq, (int32_t)nchunks, k, D, I, s, nullptr,
                                 nullptr, largest);
    // every copy has been waited on by a search (or the loop stopped): drain
    // the copy stream before it and the events go away
    (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < 2; ++i) {
        if (ready[i]) (void)hipEventDestroy(ready[i]);
        if (freed[i]) (void)hipEventDestroy(freed[i]);
    }
    if (start) (void)hipEventDestroy(start);
    (void)hipStreamDestroy(cs);
    return st;
}

extern "C" mk_status mk_debug_pool_drops(int64_t* count) {
    MK_REQUIRE(count, MK_ERR_INVALID_ARG, "null pointer");
    unsigned long long* p = nullptr;
    {
        mk_status st = mk::pool_drop_counter(&p);
        if (st != MK_OK) return st;
    }
    unsigned long long v = 0;
    MK_HIP(hipDeviceSynchronize());
    MK_HIP(hipMemcpy(&v, p, sizeof(v), hipMemcpyDeviceToHost));
    *count = (int64_t)v;
    return MK_OK;
}
