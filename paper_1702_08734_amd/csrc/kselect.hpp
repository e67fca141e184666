// Selector sizing shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mi_knn.h"

namespace mk {

constexpr int kMaxK = 1024;

// Wave-queue registers (64 entries each, a power of two) holding k entries.
inline int queue_regs(int k) {
    int r = 1;
    while (r * 64 < k) r *= 2;
    return r;
}

// Thread-queue length per wave-queue size.  Section 4.3 tunes t against k
// on Maxwell (2 for k <= 32, 3 for k <= 128, 4 for k <= 256, 8 for
// k <= 1024); here t is a power of two so that the thread-queue sort is a
// plain bitonic network on whole registers.
template <int KR>
struct SelParams;
template <> struct SelParams<1> { static constexpr int T = 2; };
template <> struct SelParams<2> { static constexpr int T = 2; };
template <> struct SelParams<4> { static constexpr int T = 4; };
template <> struct SelParams<8> { static constexpr int T = 4; };
template <> struct SelParams<16> { static constexpr int T = 8; };

// Per row, select the k best of nseg sorted lists of k keys each
// (partial[row][seg][k]) and write (score, index) pairs -- sentinel keys
// become (+inf, -1) -- or, if keys_out is given, the sorted keys themselves
// (keys_out[row][64 * queue_regs(k)], sentinel padded).  With seg_offs the
// lists of row r are seg_offs[r] .. seg_offs[r + 1] - 1 (nseg unused).  The
// second pass of the two-pass k-selection of Section 5.3.  largest: keys
// hold negated scores (largest first) and the values are emitted negated
// back, padding -inf.
mk_status merge_key_lists(const uint64_t* partial, int64_t nrows, int32_t nseg, int32_t k,
                          float* vals, int64_t* idx, hipStream_t s,
                          uint64_t* keys_out = nullptr, const int64_t* seg_offs = nullptr,
                          bool largest = false);

// Exact k-NN (knn.hip); yn may be null (then computed) for L2.
// With an arena every scratch buffer is carved from it (nothing is
// allocated); a workspace too small gives MK_ERR_UNSUPPORTED.
struct Arena;
mk_status knn_search(const float* xq, int64_t nq, const float* xb, const float* yn, int64_t nb,
                     int32_t d, int32_t k, mk_metric metric, float* D, int64_t* I,
                     hipStream_t s, Arena* arena = nullptr);
mk_status launch_norms(const float* x, int64_t n, int32_t d, float* out, hipStream_t s);

// Device address (current device) of the library's count of candidates that
// a full candidate pool of the fused kernel had to drop.  The pools are cut
// before they can overflow, so the count stays zero; it is a debug check.
mk_status pool_drop_counter(unsigned long long** out);

// Exact re-rank of candidate lists: keys[row] holds 64 * queue_regs(R) keys
// whose first R are the row's candidates (score, database row); each
// candidate is re-scored in the FP32 direct form against xb (rows of d
// floats) and the k best by (distance, row) are written to D, I.
mk_status rerank_keys(const uint64_t* keys, int64_t nq, int32_t R, const float* xq,
                      const float* xb, int32_t d, bool l2, int32_t k, float* D, int64_t* I,
                      hipStream_t s);

}  // namespace mk
