// Launch of the fused exact-search kernel for one padded dimension class DP
// (instantiated once per class in its own translation unit, knn_dNNN.hip,
// so that the many kernel variants compile in parallel).
#pragma once

#include "fused.hpp"

namespace mk {

// Candidates kept beyond k for the direct-form re-rank of the merge pass.
constexpr int kSlack = 16;

template <int KR, int DP>
mk_status knn_launch(const float* xq, int64_t nq, const float* xb, const float* yn, int64_t nb,
                     int32_t d, int32_t k, bool l2, bool vec, float* D, int64_t* I,
                     hipStream_t stream, Arena* arena) {
    using S = FusedShape<KR, DP * 4, fused_consumers<OpF32, DP>()>;
    constexpr int KS = 64 * KR;
    const int keff = k + kSlack < KS ? k + kSlack : KS;
    int64_t nqb, nchunks, chunk_len;
    plan_chunks(nq, nb, S::BQ, S::BN, KS, &nqb, &nchunks, &chunk_len);

    Scratch part, bound;
    mk_status st = part.alloc(sizeof(uint64_t) * (size_t)nq * (size_t)nchunks * S::ROW, stream, arena);
    if (st != MK_OK) return st;
    MK_TRY(bound.alloc(sizeof(uint32_t) * (size_t)bound_words(KR, nq, nchunks), stream, arena));
    if (sizing_only(arena)) return MK_OK;
    MK_TRY(clear_bounds(KR, bound.as<uint32_t>(), nq, nchunks, stream));
    const int64_t nblocks = nqb * nchunks;
    // the grid's work-item count must fit 32 bits
    MK_REQUIRE(nblocks * 64 * (kProducers + S::NC) < (1ll << 32), MK_ERR_UNSUPPORTED,
               "problem too large for one launch (search fewer queries per call)");
    unsigned long long* drops = nullptr;
    MK_TRY(pool_drop_counter(&drops));
    FusedArgs a{xq, xb, yn, nullptr, nullptr, nq, nb, d, d, chunk_len, (int32_t)nchunks,
                (int32_t)nqb, keff, part.as<uint64_t>(), bound.as<uint32_t>(), drops};
    {
        ProfScope prof("knn_fused", stream);
        auto kern = vec ? (l2 ? knn_fused<OpF32, KR, DP, true, true> : knn_fused<OpF32, KR, DP, true, false>)
                        : (l2 ? knn_fused<OpF32, KR, DP, false, true> : knn_fused<OpF32, KR, DP, false, false>);
        hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(64 * (kProducers + S::NC)), 0, stream, a);
        MK_LAUNCHED();
    }
    {
        ProfScope prof("knn_merge_rerank", stream);
        hipLaunchKernelGGL((knn_merge_rerank<KR>), dim3((unsigned)ceil_div(nq, kMergeWaves)),
                           dim3(64 * kMergeWaves), 0, stream, part.as<uint64_t>(),
                           (int32_t)nchunks, (int32_t)S::ROW, S::mem_queues ? KS : keff, xq, nq,
                           xb, d, (int32_t)vec, (int32_t)l2, k, keff, D, I);
        MK_LAUNCHED();
    }
    return MK_OK;
}

template <int DP>
mk_status knn_dispatch_k(const float* xq, int64_t nq, const float* xb, const float* yn,
                         int64_t nb, int32_t d, int32_t k, bool l2, bool vec, float* D, int64_t* I,
                         hipStream_t s, Arena* arena) {
    const int want = k + kSlack < kMaxK ? k + kSlack : kMaxK;
    switch (queue_regs(want)) {
        case 1: return knn_launch<1, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
        case 2: return knn_launch<2, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
        case 4: return knn_launch<4, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
        case 8: return knn_launch<8, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
        default: return knn_launch<16, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s, arena);
    }
}

}  // namespace mk
