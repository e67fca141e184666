// IVFADC index (Section 2 Eq. 3-6, Section 5.2-5.3): k-means training of the
// coarse quantizer and of the product quantizer, encoding and list building,
// and the search: coarse exact search (Eq. 5), query tables of term 3, the
// list scan with per-(query, list) lookup tables in LDS feeding WaveSelect,
// and the merge of the per-list partial results (Eq. 6).
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "fileio.hpp"
#include "kselect.hpp"
#include "mlp.hpp"
#include "profile.hpp"
#include "wave_select.hpp"

struct mk_ivfpq {
    int32_t d = 0, nlist = 0, M = 0, dsub = 0;
    bool trained = false;
    float* coarse = nullptr;        // [nlist, d]
    float* coarse_norms = nullptr;  // [nlist]
    float* books = nullptr;         // [M, 256, dsub]
    float* term1 = nullptr;         // [nlist, M, 256]
    int64_t ntotal = 0;
    int64_t capacity = 0;
    uint8_t* codes = nullptr;       // [capacity, M], grouped by list
    int64_t* ids = nullptr;         // [capacity]
    float* t1e = nullptr;           // [capacity] term 1 of Eq. 11 per entry
    int64_t* offsets_dev = nullptr; // [nlist + 1]
    std::vector<int64_t> offsets;   // host copy
    // scan options: 16-bit lookup tables; probed lists per scan workgroup
    // (0: chosen from the launch size, -1: all of a query's lists)
    bool lut16 = false;
    int32_t lists_per_group = 0;
};

namespace mk {

namespace {

constexpr int kBlock = 256;
// Element-wise kernels walk their items with a grid-stride loop; grids are
// capped at kMaxBlocks so that no launch exceeds the 32-bit work-item count
// of a grid dimension (a 50,000,000 x 128 array has 6.4e9 elements).
constexpr int64_t kMaxBlocks = 1 << 20;
#define kStride ((int64_t)gridDim.x * kBlock)

unsigned grid_of(int64_t n) {
    const int64_t b = ceil_div(n > 0 ? n : 1, kBlock);
    return (unsigned)(b < kMaxBlocks ? b : kMaxBlocks);
}

void free_dev(void*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <class T>
mk_status alloc_dev(T*& p, size_t count) {
    void* v = nullptr;
    MK_HIP(hipMalloc(&v, sizeof(T) * (count ? count : 1)));
    p = static_cast<T*>(v);
    return MK_OK;
}

// ---------------------------------------------------------------- k-means
__global__ void gather_rows_kernel(const float* __restrict__ src, int32_t d,
                                   const int64_t* __restrict__ rows, int64_t n,
                                   float* __restrict__ dst) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n * d; g += kStride) {
        const int64_t i = g / d, t = g % d;
        dst[g] = src[rows[i] * d + t];
    }
}

// Sum points into their centroid's FP64 accumulator (one thread per
// coordinate, so neighbouring lanes add to neighbouring addresses).
__global__ void km_accumulate(const float* __restrict__ x, int64_t n, int32_t d,
                              const int64_t* __restrict__ assign, int32_t K,
                              double* __restrict__ sums, unsigned long long* __restrict__ counts) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n * d; g += kStride) {
        const int64_t i = g / d, t = g % d;
        const int64_t a = assign[i];
        if (a < 0 || a >= K) continue;  // invalid assignments are ignored
        if (t == 0) atomicAdd(&counts[a], 1ull);
        atomicAdd(&sums[a * d + t], (double)x[g]);
    }
}

__global__ void km_finalize(const double* __restrict__ sums,
                            const unsigned long long* __restrict__ counts, int32_t K, int32_t d,
                            float* __restrict__ c, int64_t* __restrict__ counts_out) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < (int64_t)K * d;
         g += kStride) {
        const int64_t j = g / d, t = g % d;
        const unsigned long long n = counts[j];
        if (n > 0) c[g] = (float)(sums[g] / (double)n);
        if (t == 0) counts_out[j] = (int64_t)n;
    }
}

// Empty clusters, in increasing index order, split the currently largest
// cluster (ties to the lower index): multiplicative offsets 1 +- 2^-10 with
// alternating sign per coordinate, products in FP64 rounded to FP32, and the
// empty cluster takes floor(count / 2).  One workgroup walks the clusters.
__global__ __launch_bounds__(kBlock) void km_split_empty(float* __restrict__ c,
                                                         int64_t* __restrict__ counts, int32_t K,
                                                         int32_t d) {
    __shared__ int64_t s_cnt[kBlock];
    __shared__ int32_t s_idx[kBlock];
    __shared__ int32_t s_j;
    const int tid = threadIdx.x;
    int32_t j = 0;
    for (;;) {
        if (tid == 0) {
            while (j < K && counts[j] != 0) ++j;
            s_j = j;
        }
        __syncthreads();
        j = s_j;
        if (j >= K) break;
        int64_t best = -1;
        int32_t bi = 0;
        for (int32_t q = tid; q < K; q += kBlock) {
            const int64_t v = counts[q];
            if (v > best) {
                best = v;
                bi = q;
            }
        }
        s_cnt[tid] = best;
        s_idx[tid] = bi;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const int64_t o = s_cnt[tid + w];
                const int32_t oi = s_idx[tid + w];
                if (o > s_cnt[tid] || (o == s_cnt[tid] && oi < s_idx[tid])) {
                    s_cnt[tid] = o;
                    s_idx[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int32_t b = s_idx[0];
        const double eps = 1.0 / 1024.0;
        for (int32_t t = tid; t < d; t += kBlock) {
            const double s = (t % 2 == 0) ? 1.0 : -1.0;
            const double v = (double)c[(int64_t)b * d + t];
            c[(int64_t)j * d + t] = (float)(v * (1.0 + s * eps));
            c[(int64_t)b * d + t] = (float)(v * (1.0 - s * eps));
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t half = counts[b] / 2;
            counts[j] = half;
            counts[b] -= half;
        }
        __syncthreads();
        ++j;
    }
}

mk_status kmeans_update(const float* x, int64_t n, int32_t d, const int64_t* assign, int32_t K,
                        float* c, int64_t* counts_out, hipStream_t s) {
    Scratch sums, cnt, cnt64;
    MK_TRY(sums.alloc(sizeof(double) * (size_t)K * d, s));
    MK_TRY(cnt.alloc(sizeof(unsigned long long) * (size_t)K, s));
    int64_t* counts = counts_out;
    if (!counts) {
        MK_TRY(cnt64.alloc(sizeof(int64_t) * (size_t)K, s));
        counts = cnt64.as<int64_t>();
    }
    MK_HIP(hipMemsetAsync(sums.ptr, 0, sizeof(double) * (size_t)K * d, s));
    MK_HIP(hipMemsetAsync(cnt.ptr, 0, sizeof(unsigned long long) * (size_t)K, s));
    if (n > 0) {
        hipLaunchKernelGGL(km_accumulate, dim3(grid_of(n * d)), dim3(kBlock), 0,
                           s, x, n, d, assign, K, sums.as<double>(), cnt.as<unsigned long long>());
        MK_LAUNCHED();
    }
    hipLaunchKernelGGL(km_finalize, dim3(grid_of((int64_t)K * d)), dim3(kBlock),
                       0, s, sums.as<double>(), cnt.as<unsigned long long>(), K, d, c, counts);
    MK_LAUNCHED();
    hipLaunchKernelGGL(km_split_empty, dim3(1), dim3(kBlock), 0, s, c, counts, K, d);
    MK_LAUNCHED();
    return MK_OK;
}

mk_status kmeans_assign(const float* x, int64_t n, int32_t d, const float* c, int32_t K,
                        int64_t* assign, float* dist, hipStream_t s) {
    Scratch dtmp;
    float* D = dist;
    if (!D) {
        MK_TRY(dtmp.alloc(sizeof(float) * (size_t)(n > 0 ? n : 1), s));
        D = dtmp.as<float>();
    }
    return knn_search(x, n, c, nullptr, K, d, 1, MK_METRIC_L2, D, assign, s);
}

// Lloyd iterations on c [K, d], initialised by the caller.
mk_status kmeans_run(const float* x, int64_t n, int32_t d, float* c, int32_t K, int32_t niter,
                     hipStream_t s) {
    Scratch a;
    MK_TRY(a.alloc(sizeof(int64_t) * (size_t)n, s));
    for (int32_t it = 0; it < niter; ++it) {
        MK_TRY(kmeans_assign(x, n, d, c, K, a.as<int64_t>(), nullptr, s));
        MK_TRY(kmeans_update(x, n, d, a.as<int64_t>(), K, c, nullptr, s));
    }
    return MK_OK;
}

// ---------------------------------------------------------------- PQ encode
template <int DS>
__global__ __launch_bounds__(kBlock) void pq_encode_fixed(const float* __restrict__ r, int64_t n,
                                                          int32_t d, int32_t M,
                                                          const float* __restrict__ books,
                                                          uint8_t* __restrict__ codes) {
    __shared__ float cb[256 * DS];
    const int m = blockIdx.y;
    for (int e = threadIdx.x; e < 256 * DS; e += kBlock) cb[e] = books[(int64_t)m * 256 * DS + e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float rv[DS];
#pragma unroll
    for (int t = 0; t < DS; ++t) rv[t] = r[i * d + (int64_t)m * DS + t];
    float best = INFINITY;
    int arg = 0;
    for (int j = 0; j < 256; ++j) {
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < DS; ++t) {
            const float df = rv[t] - cb[j * DS + t];
            s = fmaf(df, df, s);
        }
        if (s < best) {  // strict: ties keep the lower index
            best = s;
            arg = j;
        }
    }
    codes[i * M + m] = (uint8_t)arg;
}

__global__ __launch_bounds__(kBlock) void pq_encode_any(const float* __restrict__ r, int64_t n,
                                                        int32_t d, int32_t M, int32_t ds,
                                                        const float* __restrict__ books,
                                                        uint8_t* __restrict__ codes) {
    extern __shared__ float cbs[];
    const int m = blockIdx.y;
    for (int e = threadIdx.x; e < 256 * ds; e += kBlock) cbs[e] = books[(int64_t)m * 256 * ds + e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float* rv = r + i * d + (int64_t)m * ds;
    float best = INFINITY;
    int arg = 0;
    for (int j = 0; j < 256; ++j) {
        float s = 0.f;
        for (int t = 0; t < ds; ++t) {
            const float df = rv[t] - cbs[j * ds + t];
            s = fmaf(df, df, s);
        }
        if (s < best) {
            best = s;
            arg = j;
        }
    }
    codes[i * M + m] = (uint8_t)arg;
}

mk_status pq_encode(const float* r, int64_t n, int32_t d, int32_t M, const float* books,
                    uint8_t* codes, hipStream_t s) {
    if (n == 0) return MK_OK;
    const int32_t ds = d / M;
    const dim3 grid((unsigned)ceil_div(n, kBlock), (unsigned)M), block(kBlock);
    switch (ds) {
        case 1: hipLaunchKernelGGL(pq_encode_fixed<1>, grid, block, 0, s, r, n, d, M, books, codes); break;
        case 2: hipLaunchKernelGGL(pq_encode_fixed<2>, grid, block, 0, s, r, n, d, M, books, codes); break;
        case 4: hipLaunchKernelGGL(pq_encode_fixed<4>, grid, block, 0, s, r, n, d, M, books, codes); break;
        case 8: hipLaunchKernelGGL(pq_encode_fixed<8>, grid, block, 0, s, r, n, d, M, books, codes); break;
        case 16: hipLaunchKernelGGL(pq_encode_fixed<16>, grid, block, 0, s, r, n, d, M, books, codes); break;
        default:
            hipLaunchKernelGGL(pq_encode_any, grid, block, sizeof(float) * 256 * ds, s, r, n, d, M,
                               ds, books, codes);
            break;
    }
    MK_LAUNCHED();
    return MK_OK;
}

// ---------------------------------------------------------------- helpers
// r[i] = x[i] - c[list[i]]  (FP32)
__global__ void residual_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                const float* __restrict__ c, const int64_t* __restrict__ list,
                                float* __restrict__ r) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n * d; g += kStride) {
        const int64_t i = g / d, t = g % d;
        r[g] = x[g] - c[list[i] * d + t];
    }
}

// dst[i, :] = src[i, off : off + w]
__global__ void columns_kernel(const float* __restrict__ src, int64_t n, int32_t d, int32_t off,
                               int32_t w, float* __restrict__ dst) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n * w; g += kStride) {
        const int64_t i = g / w, t = g % w;
        dst[g] = src[i * d + off + t];
    }
}

// term1[L, m, j] = ||c_{m,j}||^2 + 2 <c_L^m, c_{m,j}>   (Eq. 11, term 1)
__global__ void term1_kernel(const float* __restrict__ coarse, const float* __restrict__ books,
                             int32_t nlist, int32_t M, int32_t ds, float* __restrict__ term1) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < (int64_t)nlist * M * 256;
         g += kStride) {
        const int64_t L = g / (M * 256);
        const int32_t m = (int32_t)((g / 256) % M), j = (int32_t)(g % 256);
        const float* cw = books + ((int64_t)m * 256 + j) * ds;
        const float* cl = coarse + L * (int64_t)M * ds + (int64_t)m * ds;
        float nn = 0.f, ip = 0.f;
        for (int t = 0; t < ds; ++t) {
            nn = fmaf(cw[t], cw[t], nn);
            ip = fmaf(cl[t], cw[t], ip);
        }
        term1[g] = fmaf(2.f, ip, nn);
    }
}

// term3[q, m, j] = <x_q^m, c_{m,j}>   (Eq. 11, term 3)
// term3[q][m][j] = <x_q^m, c_{m,j}> (Eq. 11).  One workgroup per (tile of
// kT3Queries queries, sub-quantizer m), thread j owns codeword j; the
// codebook and the queries' sub-vectors pass through LDS in slices of 16
// components (summed in component order), and each query's 256 outputs are
// written as one coalesced row.
constexpr int kT3Queries = 16;

__global__ __launch_bounds__(256) void term3_kernel(const float* __restrict__ xq, int64_t nq,
                                                    int32_t M, int32_t ds,
                                                    const float* __restrict__ books,
                                                    float* __restrict__ term3) {
    __shared__ float cb[256][17];
    __shared__ float xs[kT3Queries][16];
    const int64_t q0 = (int64_t)blockIdx.x * kT3Queries;
    const int32_t m = blockIdx.y;
    const int j = threadIdx.x;
    const int d = M * ds;
    float acc[kT3Queries];
#pragma unroll
    for (int i = 0; i < kT3Queries; ++i) acc[i] = 0.f;
    for (int t0 = 0; t0 < ds; t0 += 16) {
        const int w = ds - t0 < 16 ? ds - t0 : 16;
        for (int e = j; e < 256 * 16; e += 256) {
            const int jj = e / 16, t = e % 16;
            cb[jj][t] = t < w ? books[((int64_t)m * 256 + jj) * ds + t0 + t] : 0.f;
        }
        for (int e = j; e < kT3Queries * 16; e += 256) {
            const int i = e / 16, t = e % 16;
            const int64_t q = q0 + i;
            xs[i][t] = (t < w && q < nq) ? xq[q * d + (int64_t)m * ds + t0 + t] : 0.f;
        }
        __syncthreads();
        for (int t = 0; t < w; ++t) {
            const float c = cb[j][t];
#pragma unroll
            for (int i = 0; i < kT3Queries; ++i) acc[i] = fmaf(xs[i][t], c, acc[i]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kT3Queries; ++i) {
        const int64_t q = q0 + i;
        if (q < nq) term3[(q * M + m) * 256 + j] = acc[i];
    }
}

mk_status launch_term3(const float* xq, int64_t nq, int32_t M, int32_t ds, const float* books,
                       float* term3, hipStream_t s) {
    if (nq == 0) return MK_OK;
    hipLaunchKernelGGL(term3_kernel, dim3((unsigned)ceil_div(nq, kT3Queries), (unsigned)M),
                       dim3(256), 0, s, xq, nq, M, ds, books, term3);
    MK_LAUNCHED();
    return MK_OK;
}

__global__ void fill_u32_kernel(unsigned int* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += kStride) a[i] = 0u;
}

// Stable placement of a batch into its lists without sorting.  The batch is
// cut into chunks of kPlaceChunk entries, one wave each, walked 64 entries
// at a time in batch order.  Within a group of 64 the lanes with equal lists
// are found by repeated ballots on the first remaining lane's list; the
// group's count for that list goes to the chunk's counter in one atomic.
//   place_count: cnt[c][L] = entries of chunk c in list L
//   place_prefix: per list, exclusive prefix over chunks (cnt[c][L] becomes
//                 the list rank of chunk c's first entry) and the total
//   place_new:   the same walk again; the atomic's old value plus the lane's
//                rank among equal lanes below it is the entry's rank in its
//                list among the batch, so entries keep batch order per list
constexpr int64_t kPlaceChunk = 65536;

template <bool PLACE>
__device__ __forceinline__ void place_walk(const int64_t* __restrict__ list, int64_t nb,
                                           int32_t nlist, unsigned int* __restrict__ cnt,
                                           const int64_t* __restrict__ new_off,
                                           const int64_t* __restrict__ old_off, int32_t M,
                                           const uint8_t* __restrict__ batch_codes, int64_t id0,
                                           uint8_t* __restrict__ codes, int64_t* __restrict__ ids) {
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    unsigned int* row = cnt + c * (int64_t)nlist;
    const int64_t lo = c * kPlaceChunk;
    const int64_t hi = lo + kPlaceChunk < nb ? lo + kPlaceChunk : nb;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t g = lo; g < hi; g += 64) {
        const int64_t i = g + lane;
        const bool ok = i < hi;
        const int64_t L = ok ? list[i] : -1;
        uint64_t todo = __ballot(ok);
        int64_t rank = 0;
        while (todo) {
            const int first = __builtin_ctzll(todo);
            const int64_t Lf = __shfl(L, first, 64);
            const uint64_t same = __ballot(L == Lf) & todo;
            unsigned int base = 0;
            if (lane == first) {
                if (PLACE)
                    base = atomicAdd(&row[Lf], (unsigned int)__popcll(same));
                else
                    atomicAdd(&row[Lf], (unsigned int)__popcll(same));
            }
            if (PLACE) {
                base = __shfl(base, first, 64);
                if ((same >> lane) & 1ull) rank = (int64_t)base + __popcll(same & below);
            }
            todo &= ~same;
        }
        if (PLACE && ok) {
            const int64_t pos = new_off[L] + (old_off[L + 1] - old_off[L]) + rank;
            ids[pos] = id0 + i;
            for (int m = 0; m < M; ++m) codes[pos * M + m] = batch_codes[i * M + m];
        }
    }
}

__global__ __launch_bounds__(64) void place_count_kernel(const int64_t* __restrict__ list,
                                                         int64_t nb, int32_t nlist,
                                                         unsigned int* __restrict__ cnt) {
    place_walk<false>(list, nb, nlist, cnt, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr);
}

__global__ void place_prefix_kernel(unsigned int* __restrict__ cnt, int64_t nchunks,
                                    int32_t nlist, unsigned long long* __restrict__ total) {
    const int64_t L = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (L >= nlist) return;
    unsigned long long run = 0;
    for (int64_t c = 0; c < nchunks; ++c) {
        const unsigned int v = cnt[c * nlist + L];
        cnt[c * nlist + L] = (unsigned int)run;
        run += v;
    }
    total[L] = run;
}

__global__ __launch_bounds__(64) void place_new_kernel(const int64_t* __restrict__ list,
                                                       int64_t nb, int32_t nlist,
                                                       unsigned int* __restrict__ cnt,
                                                       const int64_t* __restrict__ new_off,
                                                       const int64_t* __restrict__ old_off,
                                                       int32_t M,
                                                       const uint8_t* __restrict__ batch_codes,
                                                       int64_t id0, uint8_t* __restrict__ codes,
                                                       int64_t* __restrict__ ids) {
    place_walk<true>(list, nb, nlist, cnt, new_off, old_off, M, batch_codes, id0, codes, ids);
}

// Old entries of list L move from old_off[L] + e to new_off[L] + e.
__global__ void move_old_kernel(const int64_t* __restrict__ old_off,
                                const int64_t* __restrict__ new_off, int32_t M,
                                const uint8_t* __restrict__ old_codes,
                                const int64_t* __restrict__ old_ids, uint8_t* __restrict__ codes,
                                int64_t* __restrict__ ids) {
    const int32_t L = blockIdx.x;
    const int64_t lo = old_off[L], n = old_off[L + 1] - lo, dst = new_off[L];
    for (int64_t e = threadIdx.x; e < n; e += kBlock) {
        ids[dst + e] = old_ids[lo + e];
        for (int m = 0; m < M; ++m) codes[(dst + e) * M + m] = old_codes[(lo + e) * M + m];
    }
}

// ---------------------------------------------------------------- list scan
constexpr int kScanWaves = 4;

// One workgroup per (query, probe rank).  The list's lookup tables
// LUT[m][j] = term1[L][m][j] - 2 term3[q][m][j] are staged in LDS; each lane
// takes one code at a time (coalesced 16-byte loads when M is a multiple of
// 16), sums term2 + sum_m LUT[m][code_m] (Eq. 10 via Eq. 11) and offers it
// to its wave's selector keyed by (distance, offset in list) -- offset order
// is id order inside a list.  The four waves' queues are merged through LDS
// and the winners' ids resolved (Section 5.3: ids only for the selected).
// Probe-count features: F[q] = [xq[q] ; the kProbeDists smallest squared
// coarse distances] (cd holds ld ascending distances per query).
__global__ void probe_features_kernel(const float* __restrict__ xq, int64_t nq, int32_t d,
                                      const float* __restrict__ cd, int32_t ld,
                                      float* __restrict__ F) {
    const int32_t din = d + kProbeDists;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nq * din; e += kStride) {
        const int64_t q = e / din;
        const int t = (int)(e % din);
        F[e] = t < d ? xq[q * d + t] : cd[q * ld + (t - d)];
    }
}

// list_of[id] = inverted list holding id.
__global__ void list_of_kernel(const int64_t* __restrict__ offsets, int32_t nlist,
                               const int64_t* __restrict__ ids, int32_t* __restrict__ list_of) {
    const int32_t L = blockIdx.x;
    if (L >= nlist) return;
    for (int64_t pos = offsets[L] + threadIdx.x; pos < offsets[L + 1]; pos += blockDim.x)
        list_of[ids[pos]] = L;
}

// Probe count a query needs: 1-based rank of the list holding its nearest
// neighbour in its coarse order (ld entries per query), cap if not among
// them; target = log2 of it.
__global__ void probe_labels_kernel(const int64_t* __restrict__ ci, int32_t ld, int64_t nq,
                                    const int64_t* __restrict__ nn, const int32_t* __restrict__ list_of,
                                    int64_t ntotal, int32_t cap, float* __restrict__ target,
                                    int32_t* __restrict__ label) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int64_t id = nn[q];
    int32_t r = cap;
    if (id >= 0 && id < ntotal) {
        const int32_t L = list_of[id];
        for (int32_t p = 0; p < cap && p < ld; ++p)
            if (ci[q * ld + p] == L) { r = p + 1; break; }
    }
    target[q] = log2f((float)r);
    if (label) label[q] = r;
}

// Per-query probe counts and the scan's work plan in one workgroup:
// tau[q] = clamp(ceil(2^(yhat[q] + delta)), 1, cap) (also copied to `used`
// when given), and the exclusive prefix sums of the per-query workgroup
// counts ceil(tau / G): work[0] = 0, work[q + 1] = sum over q' <= q.
// Queries go 1024 at a time; a wave prefix sum, then one over the 16 waves'
// totals, then the running carry.
__global__ __launch_bounds__(1024) void probe_plan_kernel(const float* __restrict__ yhat,
                                                          int64_t nq, float delta, int32_t cap,
                                                          int32_t G, int32_t* __restrict__ tau,
                                                          int32_t* __restrict__ used,
                                                          int64_t* __restrict__ work) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        carry = 0;
        work[0] = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < nq; base += 1024) {
        const int64_t q = base + threadIdx.x;
        int64_t x = 0;
        if (q < nq) {
            const float t = exp2f(yhat[q] + delta);
            int32_t v = cap;
            if (t < (float)cap) v = t <= 1.f ? 1 : (int32_t)ceilf(t);
            tau[q] = v;
            if (used) used[q] = v;
            x = (v + G - 1) / G;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        if (wave == 0) {
            int64_t t = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int64_t y = __shfl_up(t, off, 64);
                if (lane >= off) t += y;
            }
            if (lane < 16) wsum[lane] = t;
        }
        __syncthreads();
        const int64_t incl = carry + (wave > 0 ? wsum[wave - 1] : 0) + x;
        if (q < nq) work[q + 1] = incl;
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl;
        __syncthreads();
    }
}

__global__ void entry_term1_kernel(const int64_t* __restrict__ offsets, int32_t M,
                                   const uint8_t* __restrict__ codes,
                                   const float* __restrict__ term1, float* __restrict__ t1e) {
    const int64_t L = blockIdx.x;
    const float* t1 = term1 + L * (int64_t)M * 256;
    for (int64_t pos = offsets[L] + threadIdx.x; pos < offsets[L + 1]; pos += blockDim.x) {
        const uint8_t* c = codes + pos * M;
        float v = 0.f;
        for (int m = 0; m < M; ++m) v += t1[m * 256 + c[m]];
        t1e[pos] = v;
    }
}

// One workgroup per (query, group of up to G probed lists).  The query's
// table -2 term3[q] (Eq. 11) is staged in LDS once for the group; each
// scanned entry's ADC distance is term 2 (the coarse distance of its list)
// + its stored term 1 + the M table lookups of its code bytes (Eq. 10-11).
// Waves take 64 entries at a time, list by list, into WaveSelect queues keyed
// (distance, id), the id being read only for entries that beat the queue's
// current threshold (Section 5.3 resolves ids only for selected entries);
// the 4 queues are merged into the group's partial list.
// Item -> (query, group): fixed probe count nprobe (= ld) when work is null,
// else query q owns items work[q] .. work[q + 1] - 1 and probes tau[q] lists.

// Lookup-table entry types: FP32, or FP16 (half the LDS and half the bytes
// per gather; each entry rounded once, sums still in FP32).
template <bool H16> struct LutT;
template <> struct LutT<false> {
    typedef float type;
    static __device__ __forceinline__ float make(float v) { return v; }
    static __device__ __forceinline__ float get(float v) { return v; }
};
template <> struct LutT<true> {
    typedef __half type;
    static __device__ __forceinline__ __half make(float v) { return __float2half_rn(v); }
    static __device__ __forceinline__ float get(__half v) { return __half2float(v); }
};

template <int KR, bool H16>
__global__ __launch_bounds__(64 * kScanWaves) void ivf_scan(
    const float* __restrict__ term3, const float* __restrict__ t1e,
    const float* __restrict__ coarse_d, const int64_t* __restrict__ coarse_i, int32_t ld,
    const int64_t* __restrict__ offsets, const uint8_t* __restrict__ codes,
    const int64_t* __restrict__ ids, int32_t M, int32_t G, int32_t k,
    uint64_t* __restrict__ part, const int64_t* __restrict__ work,
    const int32_t* __restrict__ tau, int64_t nq, int64_t excl_base) {
    constexpr int T = SelParams<KR>::T;
    typedef LutT<H16> LT;
    typedef typename LT::type lut_t;
    extern __shared__ __align__(16) unsigned char smem[];
    lut_t* lut = reinterpret_cast<lut_t*>(smem);
    uint64_t* qbuf = reinterpret_cast<uint64_t*>(smem + (size_t)M * 256 * sizeof(lut_t));

    const int64_t item = blockIdx.x;
    int64_t q, g;
    int32_t np;
    if (work) {
        if (item >= work[nq]) return;  // grid sized for the largest possible count
        int64_t lo = 0, hi = nq;  // largest q with work[q] <= item
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (work[mid] <= item) lo = mid; else hi = mid;
        }
        q = lo;
        g = item - work[q];
        np = tau[q];
    } else {
        const int64_t ng = (ld + G - 1) / G;
        q = item / ng;
        g = item - q * ng;
        np = ld;
    }
    const int32_t p0 = (int32_t)(g * G);
    const int32_t ns = np - p0 < G ? np - p0 : G;  // lists in this group
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    uint64_t* out = part + item * k;
    // k-NN graph construction: query q is node excl_base + q, not its own
    // neighbour (no exclusion when excl_base < 0; ids are >= 0)
    const int64_t excl = excl_base >= 0 ? excl_base + q : -1;

    const float* t3 = term3 + q * (int64_t)M * 256;
    for (int e = threadIdx.x; e < M * 256; e += 64 * kScanWaves) lut[e] = LT::make(-2.f * t3[e]);
    __syncthreads();

    WaveSelect<KR, T> ws;
    ws.init(k);
    const bool vec16 = (M & 15) == 0;
    const int64_t* cirow = coarse_i + q * ld + p0;
    const float* cdrow = coarse_d + q * ld + p0;
#pragma unroll 1
    for (int32_t sl = 0; sl < ns; ++sl) {
        const int64_t L = cirow[sl];
        if (L < 0) continue;  // fewer lists than probes (wave-uniform)
        const float term2 = cdrow[sl];
        const int64_t lo = offsets[L];
        const int64_t n = offsets[L + 1] - lo;
        const uint8_t* lc = codes + lo * M;
        const float* lt = t1e + lo;
        const int64_t* lid = ids + lo;
#pragma unroll 1
        for (int64_t e0 = (int64_t)wave * 64; e0 < n; e0 += 64 * kScanWaves) {
            const int64_t e = e0 + lane;
            const bool ok = e < n;
            float dist = 0.f;
            if (ok) {
                dist = term2 + lt[e];
                const uint8_t* c = lc + e * M;
                if (vec16) {
                    for (int m0 = 0; m0 < M; m0 += 16) {
                        const uint4 w = *reinterpret_cast<const uint4*>(c + m0);
                        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int m = m0 + 4 * h + b;
                                dist += LT::get(lut[m * 256 + ((ww[h] >> (8 * b)) & 0xFF)]);
                            }
                        }
                    }
                } else {
                    for (int m0 = 0; m0 < M; m0 += 4) {
                        const uint32_t w = *reinterpret_cast<const uint32_t*>(c + m0);
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            dist += LT::get(lut[(m0 + b) * 256 + ((w >> (8 * b)) & 0xFF)]);
                    }
                }
            }
            // keyed (distance, id): ids are unique, so the order is total and
            // the selected set does not depend on how lists are grouped; the
            // id is read only for an entry that can enter the queue
            uint64_t key = kSentinel;
            if (ok && ws.may_take(dist)) {
                const int64_t id = lid[e];
                if (id != excl) key = make_key(dist, (uint32_t)id);
            }
            if (ws.push(key)) ws.merge();
        }
    }
    ws.finish();

    // merge the waves' queues: each publishes its first k keys
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        if (e < k) qbuf[wave * k + e] = ws.w[r];
    }
    __syncthreads();
    if (wave == 0) {
        WaveSelect<KR, T> fin;
        fin.init(k);
        const int tot = kScanWaves * k;
#pragma unroll 1
        for (int e0 = 0; e0 < tot; e0 += 64) {
            const int e = e0 + lane;
            if (fin.push(e < tot ? qbuf[e] : kSentinel)) fin.merge();
        }
        fin.finish();
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            const int e = r * 64 + lane;
            if (e < k) out[e] = fin.w[r];
        }
    }
}

// Lists per workgroup: as many as keep the launch at 1024+ workgroups
// (about 4 per CU), so each query's table is staged once for as many lists
// as possible and fewer partial lists reach the merge; with enough queries
// every query's lists go to one workgroup (10^7 x 128, 4096 lists, k = 100:
// nprobe 128 and 10^4 queries 11.3 ms per-query against 15.6 ms for groups
// of 16; 1024 queries, nprobe 8 / 64 / 128, 0.47 / 1.41 / 2.65 ms at 2048+
// workgroups against 0.42 / 1.29 / 2.49 ms; 256 queries, nprobe 64 with
// R = 256 0.90 -> 0.85 ms, and larger groups than that slower).  Queues of
// 512+ entries aim at 512+ workgroups: each workgroup's merge of its four
// waves' queues costs more than the parallelism it buys (5*10^7 x 128,
// R = 1024, 9 probes per query: 256 queries 1.41 -> 1.15 ms with 4 lists per
// group, 1024 queries 2.31 -> 1.94 ms with all of a query's lists).
int32_t scan_group(int64_t total_probes, int32_t nprobe, int32_t k) {
    const int64_t g = total_probes / (k >= 512 ? 512 : 1024);
    return (int32_t)(g < 1 ? 1 : g > nprobe ? nprobe : g);
}

// The index's choice of lists per workgroup for nq queries probing up to
// nprobe lists each: automatic (scan_group), all of a query's lists in one
// workgroup (the per-query fused scan), or a fixed count.
int32_t scan_group_of(const mk_ivfpq* ix, int64_t nq, int32_t nprobe, int32_t auto_probes,
                      int32_t k) {
    if (ix->lists_per_group < 0) return nprobe;
    if (ix->lists_per_group > 0) return ix->lists_per_group < nprobe ? ix->lists_per_group : nprobe;
    return scan_group(nq * (int64_t)auto_probes, nprobe, k);
}

mk_status launch_scan(const float* term3, const float* t1e, const float* cd, const int64_t* ci,
                      int32_t ld, const int64_t* offsets, const uint8_t* codes,
                      const int64_t* ids, int32_t M, int64_t nq, int32_t G, int32_t k,
                      uint64_t* part, int64_t items, hipStream_t s,
                      const int64_t* work = nullptr, const int32_t* tau = nullptr,
                      int64_t excl_base = -1, bool lut16 = false) {
    if (items == 0) return MK_OK;
    MK_REQUIRE(items * 64 * kScanWaves < (1ll << 32), MK_ERR_UNSUPPORTED,
               "too many scan workgroups for one launch (search fewer queries per call)");
    const size_t shm = (size_t)M * 256 * (lut16 ? 2 : 4) + (size_t)kScanWaves * k * sizeof(uint64_t);
    MK_REQUIRE(shm <= 65536, MK_ERR_UNSUPPORTED,
               "lookup tables plus merge buffers exceed 64 KiB of LDS (reduce M or k, or use "
               "16-bit tables)");
    const dim3 grid((unsigned)items), block(64 * kScanWaves);
    ProfScope prof(lut16 ? "ivf_scan_lut16" : "ivf_scan", s);
#define MK_SCAN(KR)                                                                          \
    if (lut16)                                                                               \
        hipLaunchKernelGGL((ivf_scan<KR, true>), grid, block, shm, s, term3, t1e, cd, ci, ld, \
                           offsets, codes, ids, M, G, k, part, work, tau, nq, excl_base);    \
    else                                                                                     \
        hipLaunchKernelGGL((ivf_scan<KR, false>), grid, block, shm, s, term3, t1e, cd, ci,   \
                           ld, offsets, codes, ids, M, G, k, part, work, tau, nq, excl_base)
    switch (queue_regs(k)) {
        case 1: MK_SCAN(1); break;
        case 2: MK_SCAN(2); break;
        case 4: MK_SCAN(4); break;
        case 8: MK_SCAN(8); break;
        default: MK_SCAN(16); break;
    }
#undef MK_SCAN
    MK_LAUNCHED();
    return MK_OK;
}


mk_status build_term1(mk_ivfpq* ix, hipStream_t s) {
    free_dev(reinterpret_cast<void*&>(ix->term1));
    MK_TRY(alloc_dev(ix->term1, (size_t)ix->nlist * ix->M * 256));
    hipLaunchKernelGGL(term1_kernel, dim3(grid_of((int64_t)ix->nlist * ix->M * 256)), dim3(kBlock),
                       0, s, ix->coarse, ix->books, ix->nlist, ix->M, ix->dsub, ix->term1);
    MK_LAUNCHED();
    return launch_norms(ix->coarse, ix->nlist, ix->d, ix->coarse_norms, s);
}

void reset_lists(mk_ivfpq* ix) {
    free_dev(reinterpret_cast<void*&>(ix->codes));
    free_dev(reinterpret_cast<void*&>(ix->ids));
    free_dev(reinterpret_cast<void*&>(ix->t1e));
    ix->ntotal = 0;
    ix->capacity = 0;
    ix->offsets.assign(ix->nlist + 1, 0);
}

mk_status upload_offsets(mk_ivfpq* ix, hipStream_t s) {
    if (!ix->offsets_dev) MK_TRY(alloc_dev(ix->offsets_dev, ix->nlist + 1));
    MK_HIP(hipMemcpyAsync(ix->offsets_dev, ix->offsets.data(), sizeof(int64_t) * (ix->nlist + 1),
                          hipMemcpyHostToDevice, s));
    MK_HIP(hipStreamSynchronize(s));
    return MK_OK;
}

mk_status alloc_quantizers(mk_ivfpq* ix) {
    if (!ix->coarse) MK_TRY(alloc_dev(ix->coarse, (size_t)ix->nlist * ix->d));
    if (!ix->coarse_norms) MK_TRY(alloc_dev(ix->coarse_norms, (size_t)ix->nlist));
    if (!ix->books) MK_TRY(alloc_dev(ix->books, (size_t)ix->M * 256 * ix->dsub));
    return MK_OK;
}

mk_status train(mk_ivfpq* ix, const float* xt, int64_t nt, int32_t niter,
                const int64_t* coarse_rows, const int64_t* pq_rows, hipStream_t s) {
    const int32_t d = ix->d, nlist = ix->nlist, M = ix->M, ds = ix->dsub;
    MK_TRY(alloc_quantizers(ix));
    Scratch rows, assign, res, sub;
    MK_TRY(rows.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(nlist, 256), s));
    // coarse quantizer
    MK_HIP(hipMemcpyAsync(rows.ptr, coarse_rows, sizeof(int64_t) * nlist, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((int64_t)nlist * d)), dim3(kBlock), 0, s,
                       xt, d, rows.as<int64_t>(), (int64_t)nlist, ix->coarse);
    MK_LAUNCHED();
    MK_TRY(kmeans_run(xt, nt, d, ix->coarse, nlist, niter, s));
    // residuals of the training set to the final coarse centroids
    MK_TRY(assign.alloc(sizeof(int64_t) * (size_t)nt, s));
    MK_TRY(res.alloc(sizeof(float) * (size_t)nt * d, s));
    MK_TRY(sub.alloc(sizeof(float) * (size_t)nt * ds, s));
    MK_TRY(kmeans_assign(xt, nt, d, ix->coarse, nlist, assign.as<int64_t>(), nullptr, s));
    hipLaunchKernelGGL(residual_kernel, dim3(grid_of(nt * d)), dim3(kBlock), 0, s, xt, nt, d,
                       ix->coarse, assign.as<int64_t>(), res.as<float>());
    MK_LAUNCHED();
    // M independent sub-quantizers of 256 centroids on contiguous sub-vectors
    for (int32_t m = 0; m < M; ++m) {
        hipLaunchKernelGGL(columns_kernel, dim3(grid_of(nt * ds)), dim3(kBlock), 0, s,
                           res.as<float>(), nt, d, m * ds, ds, sub.as<float>());
        MK_LAUNCHED();
        float* cm = ix->books + (int64_t)m * 256 * ds;
        MK_HIP(hipMemcpyAsync(rows.ptr, pq_rows + (int64_t)m * 256, sizeof(int64_t) * 256,
                              hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of(256 * ds)), dim3(kBlock), 0, s,
                           sub.as<float>(), ds, rows.as<int64_t>(), (int64_t)256, cm);
        MK_LAUNCHED();
        MK_TRY(kmeans_run(sub.as<float>(), nt, ds, cm, 256, niter, s));
    }
    MK_TRY(build_term1(ix, s));
    reset_lists(ix);
    MK_TRY(upload_offsets(ix, s));
    ix->trained = true;
    return MK_OK;
}

mk_status add(mk_ivfpq* ix, const float* xb, int64_t nb, hipStream_t s) {
    const int32_t d = ix->d, nlist = ix->nlist, M = ix->M;
    if (nb == 0) return MK_OK;
    Scratch list, res, bcodes, cnt, tot, oldoff, newoff;
    MK_TRY(list.alloc(sizeof(int64_t) * nb, s));
    MK_TRY(res.alloc(sizeof(float) * nb * d, s));
    MK_TRY(bcodes.alloc((size_t)nb * M, s));
    MK_TRY(kmeans_assign(xb, nb, d, ix->coarse, nlist, list.as<int64_t>(), nullptr, s));
    hipLaunchKernelGGL(residual_kernel, dim3(grid_of(nb * d)), dim3(kBlock), 0, s, xb, nb, d,
                       ix->coarse, list.as<int64_t>(), res.as<float>());
    MK_LAUNCHED();
    MK_TRY(pq_encode(res.as<float>(), nb, d, M, ix->books, bcodes.as<uint8_t>(), s));
    // per-chunk, per-list counts of the batch, their prefix over chunks and
    // the per-list totals
    const int64_t nchunks = ceil_div(nb, kPlaceChunk);
    MK_TRY(cnt.alloc(sizeof(unsigned int) * (size_t)nchunks * nlist, s));
    MK_TRY(tot.alloc(sizeof(unsigned long long) * nlist, s));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_of(nchunks * nlist)), dim3(kBlock), 0, s,
                       cnt.as<unsigned int>(), nchunks * nlist);
    MK_LAUNCHED();
    hipLaunchKernelGGL(place_count_kernel, dim3((unsigned)nchunks), dim3(64), 0, s,
                       list.as<int64_t>(), nb, nlist, cnt.as<unsigned int>());
    MK_LAUNCHED();
    hipLaunchKernelGGL(place_prefix_kernel, dim3(grid_of(nlist)), dim3(kBlock), 0, s,
                       cnt.as<unsigned int>(), nchunks, nlist, tot.as<unsigned long long>());
    MK_LAUNCHED();
    std::vector<unsigned long long> hc(nlist);
    MK_HIP(hipMemcpyAsync(hc.data(), tot.ptr, sizeof(unsigned long long) * nlist,
                          hipMemcpyDeviceToHost, s));
    MK_HIP(hipStreamSynchronize(s));
    // new CSR offsets (host bookkeeping of nlist + 1 integers)
    std::vector<int64_t> no(nlist + 1, 0);
    for (int32_t L = 0; L < nlist; ++L)
        no[L + 1] = no[L] + (ix->offsets[L + 1] - ix->offsets[L]) + (int64_t)hc[L];
    const int64_t total = no[nlist];
    MK_REQUIRE(total < (1ll << 32) - 1, MK_ERR_UNSUPPORTED, "an index holds fewer than 2^32 - 1 vectors");
    uint8_t* ncodes = nullptr;
    int64_t* nids = nullptr;
    MK_TRY(alloc_dev(ncodes, (size_t)total * M));
    MK_TRY(alloc_dev(nids, (size_t)total));
    MK_TRY(oldoff.alloc(sizeof(int64_t) * (nlist + 1), s));
    MK_TRY(newoff.alloc(sizeof(int64_t) * (nlist + 1), s));
    MK_HIP(hipMemcpyAsync(oldoff.ptr, ix->offsets.data(), sizeof(int64_t) * (nlist + 1),
                          hipMemcpyHostToDevice, s));
    MK_HIP(hipMemcpyAsync(newoff.ptr, no.data(), sizeof(int64_t) * (nlist + 1),
                          hipMemcpyHostToDevice, s));
    if (ix->ntotal > 0) {
        hipLaunchKernelGGL(move_old_kernel, dim3(nlist), dim3(kBlock), 0, s, oldoff.as<int64_t>(),
                           newoff.as<int64_t>(), M, ix->codes, ix->ids, ncodes, nids);
        MK_LAUNCHED();
    }
    hipLaunchKernelGGL(place_new_kernel, dim3((unsigned)nchunks), dim3(64), 0, s,
                       list.as<int64_t>(), nb, nlist, cnt.as<unsigned int>(),
                       newoff.as<int64_t>(), oldoff.as<int64_t>(), M, bcodes.as<uint8_t>(),
                       ix->ntotal, ncodes, nids);
    MK_LAUNCHED();
    MK_HIP(hipStreamSynchronize(s));
    free_dev(reinterpret_cast<void*&>(ix->codes));
    free_dev(reinterpret_cast<void*&>(ix->ids));
    ix->codes = ncodes;
    ix->ids = nids;
    ix->capacity = total;
    ix->ntotal = total;
    ix->offsets = no;
    MK_TRY(upload_offsets(ix, s));
    // per-entry term 1 of Eq. 11 for the new list layout
    free_dev(reinterpret_cast<void*&>(ix->t1e));
    MK_TRY(alloc_dev(ix->t1e, (size_t)total));
    hipLaunchKernelGGL(entry_term1_kernel, dim3(nlist), dim3(kBlock), 0, s, ix->offsets_dev, M,
                       ix->codes, ix->term1, ix->t1e);
    MK_LAUNCHED();
    MK_HIP(hipStreamSynchronize(s));
    return MK_OK;
}

// Steps shared by the fixed-probe searches: the probe set and term 2 by exact
// search over the coarse centroids (Eq. 5), term 3 per query, and the list
// scan into `part` = per query `ngroups` partial lists of kk keys.
mk_status scan_fixed(mk_ivfpq* ix, const float* xq, int64_t nq, int32_t nprobe, int32_t kk,
                     Scratch& part, int64_t* ngroups, hipStream_t s, int64_t excl_base = -1) {
    const int32_t M = ix->M;
    Scratch cd, ci, t3;
    MK_TRY(cd.alloc(sizeof(float) * nq * nprobe, s));
    MK_TRY(ci.alloc(sizeof(int64_t) * nq * nprobe, s));
    MK_TRY(t3.alloc(sizeof(float) * nq * M * 256, s));
    const int32_t G = scan_group_of(ix, nq, nprobe, nprobe, kk);
    *ngroups = ceil_div(nprobe, G);
    MK_TRY(part.alloc(sizeof(uint64_t) * nq * *ngroups * kk, s));
    MK_TRY(knn_search(xq, nq, ix->coarse, ix->coarse_norms, ix->nlist, ix->d, nprobe,
                      MK_METRIC_L2, cd.as<float>(), ci.as<int64_t>(), s));
    {
        ProfScope prof("ivf_term3", s);
        MK_TRY(launch_term3(xq, nq, M, ix->dsub, ix->books, t3.as<float>(), s));
    }
    return launch_scan(t3.as<float>(), ix->t1e, cd.as<float>(), ci.as<int64_t>(), nprobe,
                       ix->offsets_dev, ix->codes, ix->ids, M, nq, G, kk, part.as<uint64_t>(),
                       nq * *ngroups, s, nullptr, nullptr, excl_base, ix->lut16);
}

mk_status search(mk_ivfpq* ix, const float* xq, int64_t nq, int32_t k, int32_t nprobe, float* D,
                 int64_t* I, hipStream_t s, int64_t excl_base = -1) {
    Scratch part;
    int64_t ng = 0;
    MK_TRY(scan_fixed(ix, xq, nq, nprobe, k, part, &ng, s, excl_base));
    ProfScope prof("ivf_merge", s);
    return merge_key_lists(part.as<uint64_t>(), nq, (int32_t)ng, k, D, I, s);
}

// IVFADC short list of R entries per query, then exact re-ranking of that
// list against the full-precision database rows (row id of xb = vector id).
mk_status search_rerank(mk_ivfpq* ix, const float* xq, int64_t nq, int32_t k, int32_t nprobe,
                        int32_t R, const float* xb, float* D, int64_t* I, hipStream_t s,
                        int64_t excl_base = -1) {
    Scratch part, keys;
    int64_t ng = 0;
    MK_TRY(scan_fixed(ix, xq, nq, nprobe, R, part, &ng, s, excl_base));
    MK_TRY(keys.alloc(sizeof(uint64_t) * nq * 64 * queue_regs(R), s));
    {
        ProfScope prof("ivf_merge", s);
        MK_TRY(merge_key_lists(part.as<uint64_t>(), nq, (int32_t)ng, R, nullptr, nullptr, s,
                               keys.as<uint64_t>()));
    }
    return rerank_keys(keys.as<uint64_t>(), nq, R, xq, xb, ix->d, true, k, D, I, s);
}

mk_status probe_features(const mk_ivfpq* ix, const float* xq, int64_t nq, float* F,
                         hipStream_t s) {
    Scratch cd, ci;
    MK_TRY(cd.alloc(sizeof(float) * nq * kProbeDists, s));
    MK_TRY(ci.alloc(sizeof(int64_t) * nq * kProbeDists, s));
    MK_TRY(knn_search(xq, nq, ix->coarse, ix->coarse_norms, ix->nlist, ix->d, kProbeDists,
                      MK_METRIC_L2, cd.as<float>(), ci.as<int64_t>(), s));
    hipLaunchKernelGGL(probe_features_kernel,
                       dim3(grid_of(nq * (ix->d + kProbeDists))), dim3(kBlock), 0, s, xq, nq,
                       ix->d, cd.as<float>(), kProbeDists, F);
    MK_LAUNCHED();
    return MK_OK;
}

mk_status probe_labels(const mk_ivfpq* ix, const float* xq, int64_t nq, const int64_t* nn,
                       int32_t cap, float* target, int32_t* label, hipStream_t s) {
    Scratch cd, ci, lof;
    MK_TRY(cd.alloc(sizeof(float) * nq * cap, s));
    MK_TRY(ci.alloc(sizeof(int64_t) * nq * cap, s));
    MK_TRY(lof.alloc(sizeof(int32_t) * (ix->ntotal > 0 ? ix->ntotal : 1), s));
    MK_TRY(knn_search(xq, nq, ix->coarse, ix->coarse_norms, ix->nlist, ix->d, cap, MK_METRIC_L2,
                      cd.as<float>(), ci.as<int64_t>(), s));
    hipLaunchKernelGGL(list_of_kernel, dim3(ix->nlist), dim3(kBlock), 0, s, ix->offsets_dev,
                       ix->nlist, ix->ids, lof.as<int32_t>());
    MK_LAUNCHED();
    hipLaunchKernelGGL(probe_labels_kernel, dim3(grid_of(nq)), dim3(kBlock), 0, s,
                       ci.as<int64_t>(), cap, nq, nn, lof.as<int32_t>(), ix->ntotal, cap, target,
                       label);
    MK_LAUNCHED();
    return MK_OK;
}

// IVFADC search with a per-query probe count predicted by the network from
// the query and its coarse distances; R > 0 adds the exact re-rank of an
// R-entry short list against xb.
mk_status search_learned(mk_ivfpq* ix, const mk_mlp* net, float delta, const float* xq,
                         int64_t nq, int32_t k, int32_t cap, int32_t R, const float* xb,
                         float* D, int64_t* I, int32_t* used, hipStream_t s) {
    const int32_t M = ix->M;
    const int32_t kk = R > 0 ? R : k;
    Scratch cd, ci, F, yhat, tau, work, t3, part, keys;
    MK_TRY(cd.alloc(sizeof(float) * nq * cap, s));
    MK_TRY(ci.alloc(sizeof(int64_t) * nq * cap, s));
    MK_TRY(F.alloc(sizeof(float) * nq * (ix->d + kProbeDists), s));
    MK_TRY(yhat.alloc(sizeof(float) * nq, s));
    MK_TRY(tau.alloc(sizeof(int32_t) * nq, s));
    MK_TRY(work.alloc(sizeof(int64_t) * (nq + 1), s));
    // coarse order up to cap probes; its first kProbeDists distances are the
    // network's distance features
    MK_TRY(knn_search(xq, nq, ix->coarse, ix->coarse_norms, ix->nlist, ix->d, cap, MK_METRIC_L2,
                      cd.as<float>(), ci.as<int64_t>(), s));
    hipLaunchKernelGGL(probe_features_kernel,
                       dim3(grid_of(nq * (ix->d + kProbeDists))), dim3(kBlock), 0, s, xq, nq,
                       ix->d, cd.as<float>(), cap, F.as<float>());
    MK_LAUNCHED();
    {
        ProfScope prof("mlp_forward", s);
        MK_TRY(mlp_forward_dev(net, F.as<float>(), nq, yhat.as<float>(), s));
    }
    // probe counts and the scan's work plan on the device: the scan grid is
    // sized for tau = cap everywhere and the surplus workgroups return at
    // once, so the search never waits for the host
    const int32_t G = scan_group_of(ix, nq, cap, cap < 8 ? cap : 8, kk);
    const int64_t max_items = nq * ceil_div(cap, G);
    hipLaunchKernelGGL(probe_plan_kernel, dim3(1), dim3(1024), 0, s, yhat.as<float>(), nq, delta,
                       cap, G, tau.as<int32_t>(), used, work.as<int64_t>());
    MK_LAUNCHED();
    MK_TRY(t3.alloc(sizeof(float) * nq * M * 256, s));
    MK_TRY(part.alloc(sizeof(uint64_t) * max_items * kk, s));
    {
        ProfScope prof("ivf_term3", s);
        MK_TRY(launch_term3(xq, nq, M, ix->dsub, ix->books, t3.as<float>(), s));
    }
    MK_TRY(launch_scan(t3.as<float>(), ix->t1e, cd.as<float>(), ci.as<int64_t>(), cap,
                       ix->offsets_dev, ix->codes, ix->ids, M, nq, G, kk, part.as<uint64_t>(),
                       max_items, s, work.as<int64_t>(), tau.as<int32_t>(), -1, ix->lut16));
    if (R <= 0) {
        ProfScope prof("ivf_merge", s);
        return merge_key_lists(part.as<uint64_t>(), nq, 0, k, D, I, s, nullptr,
                               work.as<int64_t>());
    }
    MK_TRY(keys.alloc(sizeof(uint64_t) * nq * 64 * queue_regs(R), s));
    {
        ProfScope prof("ivf_merge", s);
        MK_TRY(merge_key_lists(part.as<uint64_t>(), nq, 0, R, nullptr, nullptr, s,
                               keys.as<uint64_t>(), work.as<int64_t>()));
    }
    return rerank_keys(keys.as<uint64_t>(), nq, R, xq, xb, ix->d, true, k, D, I, s);
}

}  // namespace

}  // namespace mk

// ---------------------------------------------------------------- C ABI
extern "C" mk_status mk_kmeans_assign(const float* x, int64_t n, int32_t d, const float* c,
                                      int32_t K, int64_t* assign, float* dist,
                                      mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1 && K >= 1, MK_ERR_INVALID_ARG, "need n >= 0, d >= 1, K >= 1");
    if (n == 0) return MK_OK;
    MK_REQUIRE(x && c && assign, MK_ERR_INVALID_ARG, "null pointer");
    return mk::kmeans_assign(x, n, d, c, K, assign, dist, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_kmeans_update(const float* x, int64_t n, int32_t d, const int64_t* assign,
                                      int32_t K, float* c, int64_t* counts, mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1 && K >= 1, MK_ERR_INVALID_ARG, "need n >= 0, d >= 1, K >= 1");
    MK_REQUIRE(c && (n == 0 || (x && assign)), MK_ERR_INVALID_ARG, "null pointer");
    return mk::kmeans_update(x, n, d, assign, K, c, counts, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_pq_encode(const float* r, int64_t n, int32_t d, int32_t M,
                                  const float* codebooks, uint8_t* codes, mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1 && M >= 1 && d % M == 0 && d / M <= 64, MK_ERR_INVALID_ARG,
               "need d % M == 0 and d / M <= 64");
    if (n == 0) return MK_OK;
    MK_REQUIRE(r && codebooks && codes, MK_ERR_INVALID_ARG, "null pointer");
    return mk::pq_encode(r, n, d, M, codebooks, codes, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_create(int32_t d, int32_t nlist, int32_t M, mk_ivfpq** out) {
    MK_REQUIRE(out, MK_ERR_INVALID_ARG, "null output pointer");
    MK_REQUIRE(d >= 1 && d <= 256, MK_ERR_UNSUPPORTED, "d must be in [1, 256]");
    MK_REQUIRE(nlist >= 1 && nlist <= (1 << 24), MK_ERR_INVALID_ARG, "nlist must be in [1, 2^24]");
    MK_REQUIRE(M >= 4 && M <= 128 && M % 4 == 0, MK_ERR_UNSUPPORTED,
               "M must be a multiple of 4 in [4, 128]");
    MK_REQUIRE(d % M == 0, MK_ERR_INVALID_ARG, "d must be a multiple of M");
    mk_ivfpq* ix = new (std::nothrow) mk_ivfpq();
    MK_REQUIRE(ix, MK_ERR_OOM, "host allocation failed");
    ix->d = d;
    ix->nlist = nlist;
    ix->M = M;
    ix->dsub = d / M;
    ix->offsets.assign(nlist + 1, 0);
    *out = ix;
    return MK_OK;
}

extern "C" void mk_ivfpq_destroy(mk_ivfpq* ix) {
    if (!ix) return;
    mk::free_dev(reinterpret_cast<void*&>(ix->coarse));
    mk::free_dev(reinterpret_cast<void*&>(ix->coarse_norms));
    mk::free_dev(reinterpret_cast<void*&>(ix->books));
    mk::free_dev(reinterpret_cast<void*&>(ix->term1));
    mk::free_dev(reinterpret_cast<void*&>(ix->codes));
    mk::free_dev(reinterpret_cast<void*&>(ix->ids));
    mk::free_dev(reinterpret_cast<void*&>(ix->t1e));
    mk::free_dev(reinterpret_cast<void*&>(ix->offsets_dev));
    delete ix;
}

extern "C" mk_status mk_ivfpq_train(mk_ivfpq* ix, const float* xt, int64_t nt, int32_t niter,
                                    const int64_t* coarse_init_rows, const int64_t* pq_init_rows,
                                    mk_stream_t stream) {
    MK_REQUIRE(ix && xt && coarse_init_rows && pq_init_rows, MK_ERR_INVALID_ARG, "null pointer");
    MK_REQUIRE(nt >= ix->nlist && nt >= 256, MK_ERR_INVALID_ARG, "need nt >= nlist and nt >= 256");
    MK_REQUIRE(niter >= 0, MK_ERR_INVALID_ARG, "niter must be >= 0");
    MK_REQUIRE(nt < (1ll << 31), MK_ERR_UNSUPPORTED, "nt must be < 2^31");
    for (int32_t i = 0; i < ix->nlist; ++i)
        MK_REQUIRE(coarse_init_rows[i] >= 0 && coarse_init_rows[i] < nt, MK_ERR_INVALID_ARG,
                   "coarse init row out of range");
    for (int64_t i = 0; i < (int64_t)ix->M * 256; ++i)
        MK_REQUIRE(pq_init_rows[i] >= 0 && pq_init_rows[i] < nt, MK_ERR_INVALID_ARG,
                   "PQ init row out of range");
    return mk::train(ix, xt, nt, niter, coarse_init_rows, pq_init_rows,
                     static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_add(mk_ivfpq* ix, const float* xb, int64_t nb, mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(nb >= 0, MK_ERR_INVALID_ARG, "nb must be >= 0");
    MK_REQUIRE(nb == 0 || xb, MK_ERR_INVALID_ARG, "null pointer");
    MK_REQUIRE(ix->ntotal + nb < 0xFFFFFFFFll, MK_ERR_UNSUPPORTED,
               "an index holds fewer than 2^32 - 1 vectors");
    return mk::add(ix, xb, nb, static_cast<hipStream_t>(stream));
}

extern "C" int64_t mk_ivfpq_ntotal(const mk_ivfpq* ix) { return ix ? ix->ntotal : 0; }

extern "C" mk_status mk_ivfpq_search(mk_ivfpq* ix, const float* xq, int64_t nq, int32_t k,
                                     int32_t nprobe, float* D, int64_t* I, mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(nq >= 0, MK_ERR_INVALID_ARG, "nq must be >= 0");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= mk::kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1024");
    MK_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist && nprobe <= mk::kMaxK, MK_ERR_INVALID_ARG,
               "need 1 <= nprobe <= min(nlist, 1024)");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I, MK_ERR_INVALID_ARG, "null pointer");
    return mk::search(ix, xq, nq, k, nprobe, D, I, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_knn_graph(mk_ivfpq* ix, const float* xb, int64_t node0,
                                        int64_t nnodes, int32_t k, int32_t nprobe, int32_t R,
                                        float* D, int64_t* I, mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(node0 >= 0 && nnodes >= 0 && node0 + nnodes <= ix->ntotal, MK_ERR_INVALID_ARG,
               "nodes node0 .. node0 + nnodes - 1 must be ids of added vectors");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= mk::kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1024");
    MK_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist && nprobe <= mk::kMaxK, MK_ERR_INVALID_ARG,
               "need 1 <= nprobe <= min(nlist, 1024)");
    MK_REQUIRE(R == 0 || (R >= k && R <= mk::kMaxK), MK_ERR_INVALID_ARG,
               "R must be 0 (no re-rank) or in [k, 1024]");
    if (nnodes == 0) return MK_OK;
    MK_REQUIRE(xb && D && I, MK_ERR_INVALID_ARG, "null pointer");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // batches bound the scratch (coarse results, term 3, partial lists)
    constexpr int64_t kBatch = 32768;
    for (int64_t b = 0; b < nnodes; b += kBatch) {
        const int64_t n = nnodes - b < kBatch ? nnodes - b : kBatch;
        const int64_t first = node0 + b;
        const float* xq = xb + first * ix->d;
        if (R > 0)
            MK_TRY(mk::search_rerank(ix, xq, n, k, nprobe, R, xb, D + b * k, I + b * k, s, first));
        else
            MK_TRY(mk::search(ix, xq, n, k, nprobe, D + b * k, I + b * k, s, first));
    }
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_search_rerank(mk_ivfpq* ix, const float* xq, int64_t nq,
                                            int32_t k, int32_t nprobe, int32_t R,
                                            const float* xb, int64_t nb, float* D, int64_t* I,
                                            mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(nq >= 0, MK_ERR_INVALID_ARG, "nq must be >= 0");
    MK_REQUIRE(k >= 1 && k <= R, MK_ERR_INVALID_ARG, "need 1 <= k <= R");
    MK_REQUIRE(R <= mk::kMaxK, MK_ERR_UNSUPPORTED, "R must be <= 1024");
    MK_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist && nprobe <= mk::kMaxK, MK_ERR_INVALID_ARG,
               "need 1 <= nprobe <= min(nlist, 1024)");
    MK_REQUIRE(nb >= ix->ntotal, MK_ERR_INVALID_ARG,
               "the database must hold a row for every added id");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I && (xb || nb == 0), MK_ERR_INVALID_ARG, "null pointer");
    return mk::search_rerank(ix, xq, nq, k, nprobe, R, xb, D, I,
                             static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_probe_features(const mk_ivfpq* ix, const float* xq, int64_t nq,
                                             float* F, mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(ix->nlist >= mk::kProbeDists, MK_ERR_UNSUPPORTED, "needs nlist >= 32");
    MK_REQUIRE(nq >= 0, MK_ERR_INVALID_ARG, "nq must be >= 0");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && F, MK_ERR_INVALID_ARG, "null pointer");
    return mk::probe_features(ix, xq, nq, F, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_probe_labels(const mk_ivfpq* ix, const float* xq, int64_t nq,
                                           const int64_t* nn_ids, int32_t cap, float* target,
                                           int32_t* label, mk_stream_t stream) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(nq >= 0, MK_ERR_INVALID_ARG, "nq must be >= 0");
    MK_REQUIRE(cap >= 1 && cap <= ix->nlist && cap <= mk::kMaxK, MK_ERR_INVALID_ARG,
               "need 1 <= cap <= min(nlist, 1024)");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && nn_ids && target, MK_ERR_INVALID_ARG, "null pointer");
    return mk::probe_labels(ix, xq, nq, nn_ids, cap, target, label,
                            static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_search_learned(mk_ivfpq* ix, const mk_mlp* net, float delta,
                                             const float* xq, int64_t nq, int32_t k, int32_t cap,
                                             int32_t R, const float* xb, int64_t nb, float* D,
                                             int64_t* I, int32_t* nprobe_used,
                                             mk_stream_t stream) {
    MK_REQUIRE(ix && net, MK_ERR_INVALID_ARG, "null index or network");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_REQUIRE(mk::mlp_inputs(net) == ix->d + mk::kProbeDists, MK_ERR_INVALID_ARG,
               "network inputs must be d + 32");
    MK_REQUIRE(nq >= 0, MK_ERR_INVALID_ARG, "nq must be >= 0");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= mk::kMaxK && R <= mk::kMaxK, MK_ERR_UNSUPPORTED, "k and R must be <= 1024");
    MK_REQUIRE(cap >= mk::kProbeDists && cap <= ix->nlist && cap <= mk::kMaxK,
               MK_ERR_INVALID_ARG, "need 32 <= cap <= min(nlist, 1024)");
    MK_REQUIRE(R <= 0 || R >= k, MK_ERR_INVALID_ARG, "need R >= k for the re-rank");
    MK_REQUIRE(R <= 0 || (xb && nb >= ix->ntotal), MK_ERR_INVALID_ARG,
               "the re-rank needs a database row for every added id");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I, MK_ERR_INVALID_ARG, "null pointer");
    return mk::search_learned(ix, net, delta, xq, nq, k, cap, R, xb, D, I, nprobe_used,
                              static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_ivfpq_set_scan_options(mk_ivfpq* ix, mk_precision lut_precision,
                                               int32_t lists_per_group) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(lut_precision == MK_PREC_FP32 || lut_precision == MK_PREC_FP16, MK_ERR_UNSUPPORTED,
               "lookup tables are FP32 or FP16");
    MK_REQUIRE(lists_per_group >= -1 && lists_per_group <= mk::kMaxK, MK_ERR_INVALID_ARG,
               "lists_per_group must be -1, 0 or a count up to 1024");
    ix->lut16 = lut_precision == MK_PREC_FP16;
    ix->lists_per_group = lists_per_group;
    return MK_OK;
}

extern "C" int32_t mk_ivfpq_dim(const mk_ivfpq* ix) { return ix ? ix->d : 0; }

extern "C" mk_status mk_ivfpq_shape(const mk_ivfpq* ix, int32_t* d, int32_t* nlist, int32_t* M) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    if (d) *d = ix->d;
    if (nlist) *nlist = ix->nlist;
    if (M) *M = ix->M;
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_search_workspace_bytes(const mk_ivfpq* ix, int64_t nq, int32_t k,
                                                     int32_t nprobe, int32_t R, size_t* bytes) {
    MK_REQUIRE(ix && bytes, MK_ERR_INVALID_ARG, "null pointer");
    MK_REQUIRE(nq >= 0 && k >= 1 && nprobe >= 1, MK_ERR_INVALID_ARG, "bad sizes");
    const int64_t kk = R > 0 ? R : k;
    const int64_t qn = nq;
    // coarse search: results, and at most min(16, nlist / (8 * queue)) chunk
    // lists (the exact search's chunk plan)
    const int64_t ks = 64 * (int64_t)mk::queue_regs(std::min(nprobe + 16, mk::kMaxK));
    const int64_t chunks = std::min<int64_t>(16, std::max<int64_t>(1, ix->nlist / (8 * ks)));
    int64_t b = qn * nprobe * (4 + 8) + qn * chunks * ks * 8 + qn * 4;
    b += qn * (int64_t)ix->M * 256 * 4;      // term-3 tables
    b += qn * nprobe * kk * 8;                // per-list partial results
    if (R > 0) b += qn * 64 * (int64_t)mk::queue_regs(R) * 8;  // short lists
    b += qn * (ix->d + mk::kProbeDists) * 4 + qn * 16;          // learned-count features
    *bytes = (size_t)b;
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_get_quantizers(const mk_ivfpq* ix, float* coarse, float* codebooks) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_HIP(hipDeviceSynchronize());
    if (coarse)
        MK_HIP(hipMemcpy(coarse, ix->coarse, sizeof(float) * (size_t)ix->nlist * ix->d,
                         hipMemcpyDeviceToHost));
    if (codebooks)
        MK_HIP(hipMemcpy(codebooks, ix->books, sizeof(float) * (size_t)ix->M * 256 * ix->dsub,
                         hipMemcpyDeviceToHost));
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_set_quantizers(mk_ivfpq* ix, const float* coarse,
                                             const float* codebooks, mk_stream_t stream) {
    MK_REQUIRE(ix && coarse && codebooks, MK_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        mk_status st = mk::alloc_quantizers(ix);
        if (st != MK_OK) return st;
    }
    MK_HIP(hipMemcpyAsync(ix->coarse, coarse, sizeof(float) * (size_t)ix->nlist * ix->d,
                          hipMemcpyHostToDevice, s));
    MK_HIP(hipMemcpyAsync(ix->books, codebooks, sizeof(float) * (size_t)ix->M * 256 * ix->dsub,
                          hipMemcpyHostToDevice, s));
    mk_status st = mk::build_term1(ix, s);
    if (st != MK_OK) return st;
    mk::reset_lists(ix);
    st = mk::upload_offsets(ix, s);
    if (st != MK_OK) return st;
    ix->trained = true;
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_get_lists(const mk_ivfpq* ix, int64_t* offsets, uint8_t* codes,
                                        int64_t* ids) {
    MK_REQUIRE(ix, MK_ERR_INVALID_ARG, "null index");
    MK_HIP(hipDeviceSynchronize());
    if (offsets) std::memcpy(offsets, ix->offsets.data(), sizeof(int64_t) * (ix->nlist + 1));
    if (codes && ix->ntotal)
        MK_HIP(hipMemcpy(codes, ix->codes, (size_t)ix->ntotal * ix->M, hipMemcpyDeviceToHost));
    if (ids && ix->ntotal)
        MK_HIP(hipMemcpy(ids, ix->ids, sizeof(int64_t) * ix->ntotal, hipMemcpyDeviceToHost));
    return MK_OK;
}

// ---------------------------------------------------------------- save / load
namespace mk {
namespace {
constexpr char kIndexMagic[8] = {'M', 'K', 'I', 'V', 'F', 'P', 'Q', '\0'};
constexpr uint32_t kIndexVersion = 1;

// Fills a freshly created index from the body of an index file (after the
// header) and rebuilds the derived tables with the same kernels as
// train/add, so searches after a load equal searches before the save.
mk_status load_body(mk_ivfpq* ix, BinFile& f, int64_t ntotal, hipStream_t s) {
    const int32_t nlist = ix->nlist, M = ix->M;
    MK_TRY(alloc_quantizers(ix));
    MK_TRY(get_device(f, ix->coarse, sizeof(float) * (size_t)nlist * ix->d));
    MK_TRY(get_device(f, ix->books, sizeof(float) * (size_t)M * 256 * ix->dsub));
    std::vector<int64_t> offs(nlist + 1);
    MK_REQUIRE(f.get(offs.data(), sizeof(int64_t) * offs.size()), MK_ERR_INVALID_ARG,
               f.path + " is truncated");
    MK_REQUIRE(offs[0] == 0 && offs[nlist] == ntotal, MK_ERR_INVALID_ARG,
               f.path + ": list offsets do not span the stored entries");
    for (int32_t L = 0; L < nlist; ++L)
        MK_REQUIRE(offs[L + 1] >= offs[L], MK_ERR_INVALID_ARG, f.path + ": list offsets decrease");
    MK_TRY(alloc_dev(ix->codes, (size_t)ntotal * M));
    MK_TRY(alloc_dev(ix->ids, (size_t)ntotal));
    MK_TRY(get_device(f, ix->codes, (size_t)ntotal * M));
    MK_TRY(get_device(f, ix->ids, sizeof(int64_t) * (size_t)ntotal));
    MK_REQUIRE(f.at_end(), MK_ERR_INVALID_ARG, f.path + " has trailing bytes");
    MK_TRY(build_term1(ix, s));
    ix->offsets = offs;
    ix->ntotal = ntotal;
    ix->capacity = ntotal;
    MK_TRY(upload_offsets(ix, s));
    MK_TRY(alloc_dev(ix->t1e, (size_t)(ntotal > 0 ? ntotal : 1)));
    hipLaunchKernelGGL(entry_term1_kernel, dim3(nlist), dim3(kBlock), 0, s, ix->offsets_dev, M,
                       ix->codes, ix->term1, ix->t1e);
    MK_LAUNCHED();
    MK_HIP(hipStreamSynchronize(s));
    ix->trained = true;
    return MK_OK;
}
}  // namespace
}  // namespace mk

extern "C" mk_status mk_ivfpq_save(const mk_ivfpq* ix, const char* path) {
    MK_REQUIRE(ix && path, MK_ERR_INVALID_ARG, "null pointer");
    MK_REQUIRE(ix->trained, MK_ERR_STATE, "index is not trained");
    MK_HIP(hipDeviceSynchronize());
    mk::BinFile f(path, "wb");
    MK_REQUIRE(f.ok(), MK_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
    const bool head = f.put(mk::kIndexMagic, 8) && f.put_v(mk::kIndexVersion) && f.put_v(ix->d) &&
                      f.put_v(ix->nlist) && f.put_v(ix->M) && f.put_v(ix->ntotal);
    MK_REQUIRE(head, MK_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
    MK_TRY(mk::put_device(f, ix->coarse, sizeof(float) * (size_t)ix->nlist * ix->d));
    MK_TRY(mk::put_device(f, ix->books, sizeof(float) * (size_t)ix->M * 256 * ix->dsub));
    MK_REQUIRE(f.put(ix->offsets.data(), sizeof(int64_t) * (ix->nlist + 1)), MK_ERR_INVALID_ARG,
               std::string("write to ") + path + " failed");
    MK_TRY(mk::put_device(f, ix->codes, (size_t)ix->ntotal * ix->M));
    MK_TRY(mk::put_device(f, ix->ids, sizeof(int64_t) * (size_t)ix->ntotal));
    MK_REQUIRE(f.close(), MK_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
    return MK_OK;
}

extern "C" mk_status mk_ivfpq_load(const char* path, mk_ivfpq** out) {
    MK_REQUIRE(path && out, MK_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    mk::BinFile f(path, "rb");
    MK_REQUIRE(f.ok(), MK_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    uint32_t version = 0;
    int32_t d = 0, nlist = 0, M = 0;
    int64_t ntotal = 0;
    const bool head = f.get(magic, 8) && f.get_v(version) && f.get_v(d) && f.get_v(nlist) &&
                      f.get_v(M) && f.get_v(ntotal);
    MK_REQUIRE(head && std::memcmp(magic, mk::kIndexMagic, 8) == 0, MK_ERR_INVALID_ARG,
               std::string(path) + " is not an IVFPQ index file");
    MK_REQUIRE(version == mk::kIndexVersion, MK_ERR_UNSUPPORTED,
               std::string(path) + ": unknown index file version");
    MK_REQUIRE(ntotal >= 0 && ntotal < 0xFFFFFFFFll, MK_ERR_INVALID_ARG,
               std::string(path) + ": bad entry count");
    mk_ivfpq* ix = nullptr;
    MK_TRY(mk_ivfpq_create(d, nlist, M, &ix));
    const mk_status st = mk::load_body(ix, f, ntotal, nullptr);
    if (st != MK_OK) {
        mk_ivfpq_destroy(ix);
        return st;
    }
    *out = ix;
    return MK_OK;
}
