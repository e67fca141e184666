// Low-precision brute force with exact re-rank: the q.y term on BF16 or
// OCP-E4M3 FP8 matrix cores with FP32 accumulation selects rerank_R
// candidates per query (fused with the selection as in the FP32 path), whose
// distances are then recomputed from the FP32 rows in the direct form and
// re-ranked to the final k.  The paper computes distances in FP32 only
// (Section 2); this is the reduced-precision variant of its exact search.
#include <cmath>

#include "fused.hpp"

namespace mk {

namespace {

inline int32_t lowp_stride(int32_t d) { return (d + 15) / 16 * 16; }

inline int elem_bytes(int32_t prec) { return prec == 1 ? 2 : 1; }

// BF16 by round-to-nearest-even of the FP32 bits.
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One wave per row: BF16 copy, or FP8 copy of the row scaled by the power of
// two s with max|x| s in (224, 448] (s = 1 for an all-zero row), writing
// 1/s.  Padding elements up to the stride are zero.
template <int PREC>
__global__ __launch_bounds__(256) void quantize_rows_kernel(const float* __restrict__ x, int64_t n,
                                                            int32_t d, int32_t ld,
                                                            void* __restrict__ out,
                                                            float* __restrict__ inv_scale) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (row >= n) return;
    const float* xr = x + row * d;
    if constexpr (PREC == 1) {
        uint16_t* o = static_cast<uint16_t*>(out) + row * ld;
        for (int t = lane; t < ld; t += 64) o[t] = t < d ? to_bf16(xr[t]) : (uint16_t)0;
        if (inv_scale && lane == 0) inv_scale[row] = 1.f;
    } else {
        float m = 0.f;
        for (int t = lane; t < d; t += 64) m = fmaxf(m, fabsf(xr[t]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        // s = the largest power of two with m s <= 448 = 1.75 * 2^8, from the
        // bits of m = f 2^e (f in [1, 2)): 2^(8-e) when f <= 1.75, else
        // 2^(7-e); either way m s lands in (224, 448].  s is capped at 2^126
        // (rows with max |x| under 2^-118, subnormal ones included, keep m s
        // below 224) so that s and 1/s are normal floats built exactly from
        // their exponent fields.
        float s = 1.f, inv = 1.f;
        if (m > 0.f) {
            const uint32_t bits = __float_as_uint(m);
            const int field = (int)((bits >> 23) & 0xFF);
            int p = 126;
            if (field > 0) {
                const uint32_t frac = bits & 0x7FFFFF;  // f = 1 + frac 2^-23
                p = (frac <= 0x600000u ? 8 : 7) - (field - 127);  // 0x600000: f = 1.75
                p = p > 126 ? 126 : p;
            }
            s = __uint_as_float((uint32_t)(p + 127) << 23);
            inv = __uint_as_float((uint32_t)(127 - p) << 23);
        }
        uint16_t* o = reinterpret_cast<uint16_t*>(static_cast<uint8_t*>(out) + row * ld);
        for (int t2 = lane; 2 * t2 < ld; t2 += 64) {
            const int t = 2 * t2;
            const float a = t < d ? xr[t] * s : 0.f;
            const float b = t + 1 < d ? xr[t + 1] * s : 0.f;
            o[t2] = (uint16_t)(__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFF);
        }
        if (inv_scale && lane == 0) inv_scale[row] = inv;
    }
}

mk_status quantize(const float* x, int64_t n, int32_t d, int32_t prec, void* out, float* inv,
                   hipStream_t s) {
    if (n == 0) return MK_OK;
    const int32_t ld = lowp_stride(d);
    const size_t esize = prec == 1 ? 2 : 1;
    // launches of at most 2^24 rows (2^30 work-items: under the 32-bit
    // work-item count of a grid dimension)
    constexpr int64_t kRows = 1ll << 24;
    for (int64_t r0 = 0; r0 < n; r0 += kRows) {
        const int64_t m = n - r0 < kRows ? n - r0 : kRows;
        const dim3 grid((unsigned)ceil_div(m, 4)), block(256);
        const float* xr = x + r0 * d;
        void* o = static_cast<unsigned char*>(out) + (size_t)r0 * ld * esize;
        float* iv = inv ? inv + r0 : nullptr;
        if (prec == 1)
            hipLaunchKernelGGL(quantize_rows_kernel<1>, grid, block, 0, s, xr, m, d, ld, o, iv);
        else
            hipLaunchKernelGGL(quantize_rows_kernel<2>, grid, block, 0, s, xr, m, d, ld, o, iv);
        MK_LAUNCHED();
    }
    return MK_OK;
}

template <class Op, int KR, int DP>
mk_status lowp_launch(const float* xq, const void* xq_lp, const float* xq_inv, int64_t nq,
                      const float* xb, const void* xb_lp, const float* xb_inv, const float* yn,
                      int64_t nb, int32_t d, int32_t k, int32_t R, bool l2, float* D, int64_t* I,
                      hipStream_t stream) {
    using S = FusedShape<KR, DP * Op::BYTES, fused_consumers<Op, DP>()>;
    constexpr int KS = 64 * KR;
    int64_t nqb, nchunks, chunk_len;
    plan_chunks(nq, nb, S::BQ, S::BN, KS, &nqb, &nchunks, &chunk_len);
    Scratch part, bound;
    mk_status st = part.alloc(sizeof(uint64_t) * (size_t)nq * (size_t)nchunks * S::ROW, stream);
    if (st != MK_OK) return st;
    MK_TRY(bound.alloc(sizeof(uint32_t) * (size_t)bound_words(KR, nq, nchunks), stream));
    MK_TRY(clear_bounds(KR, bound.as<uint32_t>(), nq, nchunks, stream));
    const int64_t nblocks = nqb * nchunks;
    // the grid's work-item count must fit 32 bits
    MK_REQUIRE(nblocks * 64 * (kProducers + S::NC) < (1ll << 32), MK_ERR_UNSUPPORTED,
               "problem too large for one launch (search fewer queries per call)");
    const int32_t ld = lowp_stride(d);
    unsigned long long* drops = nullptr;
    MK_TRY(pool_drop_counter(&drops));
    FusedArgs a{xq_lp, xb_lp, yn, xq_inv, xb_inv, nq, nb, ld, ld, chunk_len, (int32_t)nchunks,
                (int32_t)nqb, R, part.as<uint64_t>(), bound.as<uint32_t>(), drops};
    {
        ProfScope prof(Op::SCALED ? "knn_fused_fp8" : "knn_fused_bf16", stream);
        auto kern = l2 ? knn_fused<Op, KR, DP, true, true> : knn_fused<Op, KR, DP, true, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(64 * (kProducers + S::NC)), 0,
                           stream, a);
        MK_LAUNCHED();
    }
    const bool vec = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(xq) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(xb) % 16 == 0);
    {
        ProfScope prof("knn_merge_rerank", stream);
        hipLaunchKernelGGL((knn_merge_rerank<KR>), dim3((unsigned)ceil_div(nq, kMergeWaves)),
                           dim3(64 * kMergeWaves), 0, stream, part.as<uint64_t>(),
                           (int32_t)nchunks, (int32_t)S::ROW, S::mem_queues ? KS : R, xq, nq, xb,
                           d, (int32_t)vec, (int32_t)l2, k, R, D, I);
        MK_LAUNCHED();
    }
    return MK_OK;
}

template <class Op, int DP>
mk_status lowp_dispatch_k(const float* xq, const void* xq_lp, const float* xq_inv, int64_t nq,
                          const float* xb, const void* xb_lp, const float* xb_inv,
                          const float* yn, int64_t nb, int32_t d, int32_t k, int32_t R, bool l2,
                          float* D, int64_t* I, hipStream_t s) {
    switch (queue_regs(R)) {
        case 1: return lowp_launch<Op, 1, DP>(xq, xq_lp, xq_inv, nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        case 2: return lowp_launch<Op, 2, DP>(xq, xq_lp, xq_inv, nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        case 4: return lowp_launch<Op, 4, DP>(xq, xq_lp, xq_inv, nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        case 8: return lowp_launch<Op, 8, DP>(xq, xq_lp, xq_inv, nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        default: return lowp_launch<Op, 16, DP>(xq, xq_lp, xq_inv, nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
    }
}

mk_status search_lowp(const float* xq, int64_t nq, const float* xb, const void* xb_lp,
                      const float* xb_inv, const float* yn_in, int64_t nb, int32_t d, int32_t k,
                      int32_t R, mk_metric metric, int32_t prec, float* D, int64_t* I,
                      hipStream_t s) {
    const bool l2 = metric == MK_METRIC_L2;
    const int32_t ld = lowp_stride(d);
    Scratch qlp, qinv, norms;
    MK_TRY(qlp.alloc((size_t)nq * ld * elem_bytes(prec), s));
    MK_TRY(qinv.alloc(sizeof(float) * (size_t)nq, s));
    MK_TRY(quantize(xq, nq, d, prec, qlp.ptr, qinv.as<float>(), s));
    const float* yn = yn_in;
    if (l2 && !yn && nb > 0) {
        MK_TRY(norms.alloc(sizeof(float) * (size_t)nb, s));
        MK_TRY(launch_norms(xb, nb, d, norms.as<float>(), s));
        yn = norms.as<float>();
    }
    if (prec == 1) {
        if (ld <= 32) return lowp_dispatch_k<OpBF16, 32>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        if (ld <= 64) return lowp_dispatch_k<OpBF16, 64>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        if (ld <= 96) return lowp_dispatch_k<OpBF16, 96>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        if (ld <= 128) return lowp_dispatch_k<OpBF16, 128>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
        return lowp_dispatch_k<OpBF16, 256>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
    }
    if (ld <= 64) return lowp_dispatch_k<OpFP8, 64>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
    if (ld <= 128) return lowp_dispatch_k<OpFP8, 128>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
    return lowp_dispatch_k<OpFP8, 256>(xq, qlp.ptr, qinv.as<float>(), nq, xb, xb_lp, xb_inv, yn, nb, d, k, R, l2, D, I, s);
}

}  // namespace

}  // namespace mk

extern "C" int32_t mk_lowp_stride(int32_t d) { return mk::lowp_stride(d); }

extern "C" mk_status mk_quantize_rows(const float* x, int64_t n, int32_t d, int32_t prec,
                                      void* out, float* inv_scales, mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1, MK_ERR_INVALID_ARG, "need n >= 0 and d >= 1");
    MK_REQUIRE(prec == MK_PREC_BF16 || prec == MK_PREC_FP8E4M3, MK_ERR_INVALID_ARG,
               "precision must be BF16 or FP8-E4M3");
    MK_REQUIRE(d <= 256, MK_ERR_UNSUPPORTED, "d must be <= 256");
    if (n == 0) return MK_OK;
    MK_REQUIRE(x && out && (inv_scales || prec == MK_PREC_BF16), MK_ERR_INVALID_ARG,
               "null pointer");
    return mk::quantize(x, n, d, prec, out, inv_scales, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_knn_search_lowp(const float* xq, int64_t nq, const float* xb,
                                        const void* xb_lp, const float* xb_inv, const float* yn,
                                        int64_t nb, int32_t d, int32_t k, int32_t rerank_R,
                                        mk_metric metric, int32_t prec, float* D, int64_t* I,
                                        mk_stream_t stream) {
    MK_REQUIRE(nq >= 0 && nb >= 0, MK_ERR_INVALID_ARG, "nq and nb must be >= 0");
    MK_REQUIRE(d >= 1, MK_ERR_INVALID_ARG, "d must be >= 1");
    MK_REQUIRE(d <= 256, MK_ERR_UNSUPPORTED, "d must be <= 256");
    MK_REQUIRE(k >= 1 && rerank_R >= k, MK_ERR_INVALID_ARG, "need 1 <= k <= rerank_R");
    MK_REQUIRE(rerank_R <= mk::kMaxK, MK_ERR_UNSUPPORTED, "rerank_R must be <= 1024");
    MK_REQUIRE(nb < (1ll << 31), MK_ERR_UNSUPPORTED, "nb must be < 2^31");
    MK_REQUIRE(metric == MK_METRIC_L2 || metric == MK_METRIC_IP, MK_ERR_INVALID_ARG, "bad metric");
    MK_REQUIRE(prec == MK_PREC_BF16 || prec == MK_PREC_FP8E4M3, MK_ERR_INVALID_ARG,
               "precision must be BF16 or FP8-E4M3");
    if (nq == 0) return MK_OK;
    MK_REQUIRE(xq && D && I && (nb == 0 || (xb && xb_lp && (xb_inv || prec == MK_PREC_BF16))),
               MK_ERR_INVALID_ARG, "null pointer");
    return mk::search_lowp(xq, nq, xb, xb_lp, xb_inv, yn, nb, d, k, rerank_R, metric, prec, D, I,
                           static_cast<hipStream_t>(stream));
}
