// Exact k-NN search (Section 2 Eq. 1-2, Section 5.1).
//
// Layout of one call:
//   1. norms: ||y||^2 per database row (one pass, Eq. 2), skipped for inner
//      products or when the caller supplies them;
//   2. knn_fused: the grid is (query block) x (database chunk).  Producer
//      waves keep their queries' MFMA A-operands in registers, stream the
//      chunk in tiles of 64 rows (prefetching the next tile's rows into
//      registers), compute the q.y tile with v_mfma_f32_16x16x4f32 and stage
//      scores (||y||^2 - 2 q.y for L2, -q.y for inner products; ||x||^2 is
//      constant per query and not needed to rank, Section 5.1) in LDS;
//      consumer waves feed them to register-resident selectors -- distance
//      computation and k-selection in one kernel, so the distance matrix
//      never reaches HBM;
//   3. knn_merge_rerank: one wave per query selects the best of the chunks'
//      partial lists (the second pass of Section 5.3's two-pass selection),
//      recomputes the kept candidates' distances in the direct form in FP32,
//      and re-ranks them.  The selection keeps k + 16 candidates (when the
//      1024-entry queue allows) so that the FP32 cancellation of the norm
//      decomposition cannot push a true neighbour out of the final k.
#include "common.hpp"
#include "kselect.hpp"
#include "profile.hpp"
#include "wave_select.hpp"

namespace mk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kSlack = 16;

// ---------------------------------------------------------------- norms
__global__ __launch_bounds__(256) void norms_kernel(const float* __restrict__ x, int64_t n,
                                                    int32_t d, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* p = x + i * d;
    float s = 0.f;
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        for (int t = 0; t < d; t += 4) {
            float4 v = *reinterpret_cast<const float4*>(p + t);
            s = fmaf(v.x, v.x, s);
            s = fmaf(v.y, v.y, s);
            s = fmaf(v.z, v.z, s);
            s = fmaf(v.w, v.w, s);
        }
    } else {
        for (int t = 0; t < d; ++t) s = fmaf(p[t], p[t], s);
    }
    out[i] = s;
}

mk_status launch_norms(const float* x, int64_t n, int32_t d, float* out, hipStream_t s) {
    if (n == 0) return MK_OK;
    hipLaunchKernelGGL(norms_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, n, d, out);
    MK_LAUNCHED();
    return MK_OK;
}

// ---------------------------------------------------------------- selectors
// QW independent selectors held by one wave (one per query the wave owns).
// Merges run one query at a time through a working copy so that the merge
// network is emitted once, not once per query.
template <int KR, int T, int QW>
struct MultiSelect {
    uint64_t w[QW][KR];
    uint64_t tq[QW][T];
    uint64_t kth[QW];
    float kth_f[QW];
    int keff;

    __device__ __forceinline__ void init(int k_eff) {
        keff = k_eff;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
#pragma unroll
            for (int r = 0; r < KR; ++r) w[q][r] = kSentinel;
#pragma unroll
            for (int i = 0; i < T; ++i) tq[q][i] = kSentinel;
            kth[q] = kSentinel;
            kth_f[q] = INFINITY;
        }
    }

    __device__ __forceinline__ void merge_slot(int q) {
        uint64_t ww[KR], tt[T];
#pragma unroll
        for (int r = 0; r < KR; ++r) ww[r] = opaque(w[0][r]);
#pragma unroll
        for (int i = 0; i < T; ++i) tt[i] = opaque(tq[0][i]);
#pragma unroll
        for (int qq = 1; qq < QW; ++qq) {
            const bool hit = qq == q;
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                const uint64_t e = opaque(w[qq][r]);
                ww[r] = hit ? e : ww[r];
            }
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const uint64_t e = opaque(tq[qq][i]);
                tt[i] = hit ? e : tt[i];
            }
        }
        ws_merge<KR, T>(ww, tt);
        const uint64_t kk = ws_element<KR>(ww, keff - 1);
        const float kf = kk == kSentinel ? INFINITY : key_score(kk);
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) {
            const bool hit = qq == q;
#pragma unroll
            for (int r = 0; r < KR; ++r) w[qq][r] = hit ? opaque(ww[r]) : w[qq][r];
#pragma unroll
            for (int i = 0; i < T; ++i) tq[qq][i] = hit ? kSentinel : tq[qq][i];
            kth[qq] = hit ? kk : kth[qq];
            kth_f[qq] = hit ? kf : kth_f[qq];
        }
    }

    // Offer, for every query q, this lane's candidate (score[q], idx); ok
    // false means no candidate.  A query whose scores all lose to its current
    // k-th score is skipped after one compare per lane.
    __device__ __forceinline__ void offer(const float (&score)[QW], uint32_t idx, bool ok) {
        uint32_t full = 0;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            if (__any(ok && score[q] <= kth_f[q])) {
                const uint64_t key = ok ? make_key(score[q], idx) : kSentinel;
                const bool take = key < kth[q];
                if (__any(take)) {
                    tq_push<T>(tq[q], key, take);
                    if (__any(tq_full<T>(tq[q]))) full |= 1u << q;
                }
            }
        }
        while (full) {
            const int q = __builtin_ctz(full);
            full &= full - 1;
            merge_slot(q);
        }
    }

    __device__ __forceinline__ void finish() {
#pragma unroll 1
        for (int q = 0; q < QW; ++q) merge_slot(q);
    }
};

__device__ __forceinline__ float4 load4_guard(const float* __restrict__ row, int dim, int d,
                                              bool vec, bool ok) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!ok) return v;
    if (vec) {
        if (dim < d) v = *reinterpret_cast<const float4*>(row + dim);
    } else {
        if (dim < d) v.x = row[dim];
        if (dim + 1 < d) v.y = row[dim + 1];
        if (dim + 2 < d) v.z = row[dim + 2];
        if (dim + 3 < d) v.w = row[dim + 3];
    }
    return v;
}

// Map hardware workgroup ids (dispatched round-robin over the 8 XCDs) to
// logical ids so that each XCD runs a contiguous logical range: the
// workgroups sharing an XCD's L2 then walk the same database chunk.
__device__ __forceinline__ int64_t xcd_logical_id(int64_t bid, int64_t nblocks) {
    const int64_t x = bid & 7, pos = bid >> 3;
    const int64_t base = nblocks >> 3, rem = nblocks & 7;
    return x * base + (x < rem ? x : rem) + pos;
}

// Workgroup of the fused kernel: 4 producer waves (one per SIMD) compute the
// q.y tile of BQ queries x BN = 64 database rows per step with
// v_mfma_f32_16x16x4f32 and write scores into one of two LDS slots, while 4
// consumer waves (one per SIMD) run the selectors of the previous step's
// tile from the other slot -- matrix cores and VALU selection overlap, one
// barrier per step.  Each producer owns QPB query blocks x DPB database
// blocks of 16 (a 4-producer grid of QG x DG), each consumer QW = BQ/NC
// queries.  Sizes per wave-queue length KR and padded dimension DP:
//   KR <= 2: BQ 64 (QW 16); KR = 4: BQ 32 (QW 8); KR >= 8 or DP > 128: BQ 16
//   (QW 4, or QW 2 over 8 consumer waves for KR = 16).
constexpr int kProducers = 4;

template <int KR, int DP>
struct FusedShape {
    // 1024-entry queues: 8 consumer waves of 2 queries (the state of four
    // 1024-entry selectors does not fit one wave's registers)
    static constexpr int NC = KR >= 16 ? 8 : 4;
    // thread-queue length: 4 for 1024-entry queues so that two selectors and
    // a working copy fit a consumer's registers
    static constexpr int T = KR >= 16 ? 4 : SelParams<KR>::T;
    static constexpr bool wide = DP > 128;
    static constexpr int QPB = (!wide && KR <= 2) ? 2 : 1;
    static constexpr int DPB = (!wide && KR <= 4) ? 2 : 1;
    static constexpr int DG = DPB == 2 ? 2 : 4;
    static constexpr int QG = kProducers / DG;
    static constexpr int BQ = QG * QPB * 16;
    static constexpr int BN = DG * DPB * 16;
    static constexpr int QW = BQ / NC;
    static_assert(BN == 64, "consumers take one column per lane");
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

template <int KR, int DP, bool VEC, bool L2>
__global__ __launch_bounds__(64 * (kProducers + FusedShape<KR, DP>::NC))
__attribute__((amdgpu_waves_per_eu(2, 2))) void knn_fused(
    const float* __restrict__ xq, int64_t nq, const float* __restrict__ xb,
    const float* __restrict__ yn, int64_t nb, int32_t d,
    int64_t chunk_len, int32_t nchunks, int32_t nqb, int32_t keff, uint64_t* __restrict__ part) {
    using S = FusedShape<KR, DP>;
    constexpr int T = S::T;
    constexpr int BQ = S::BQ, BN = S::BN, QW = S::QW, QPB = S::QPB, DPB = S::DPB, DG = S::DG;
    constexpr int LDP = BN + 4;
    constexpr int S4 = DP / 16;
    constexpr int KS = 64 * KR;
    // Database tile in LDS: BN rows of DP floats as 16-byte granules, GR per
    // row; granule c of row j is stored at position c ^ (j & SW) so that the
    // 16 rows read by one MFMA operand load fall in different banks.
    constexpr int GR = DP / 4;
    constexpr int SW = (GR % 16 == 0) ? 15 : 7;
    constexpr int NI = BN * GR / 64;  // 64-lane granule loads per tile

    __shared__ __align__(16) float btile[2][BN * DP];
    __shared__ float scores[2][BQ * LDP];

    const int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)nqb * nchunks);
    const int64_t chunk = logical / nqb;
    const int64_t qblk = logical % nqb;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t q0 = qblk * BQ;
    const int64_t c0 = chunk * chunk_len;
    const int64_t c1 = c0 + chunk_len < nb ? c0 + chunk_len : nb;
    const int64_t nsteps = c1 > c0 ? (c1 - c0 + BN - 1) / BN : 0;

    // Load the tile of rows [t0, t0 + BN) into btile[buf]; producers share
    // the NI granule loads.  Rows past the chunk repeat its last row and
    // granules past d repeat granule 0: both only ever meet zero A
    // components or unconsumed score columns.
    auto load_tile = [&](int64_t t0, int buf) {
        for (int i = wave; i < NI; i += kProducers) {
            const int g = i * 64 + lane;
            const int j = g / GR;
            const int c = (g % GR) ^ (j & SW);
            int64_t row = t0 + j;
            row = row < c1 ? row : c1 - 1;
            const int col = 4 * c < d ? 4 * c : 0;
            const float* src = xb + row * d + col;
            float* dst = &btile[buf][i * 256];  // 64 lanes x 4 floats
            if constexpr (VEC) {
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)dst, 16, 0, 0);
            } else {
                float4 v;
                v.x = col + 0 < d ? src[0] : 0.f;
                v.y = col + 1 < d ? src[1] : 0.f;
                v.z = col + 2 < d ? src[2] : 0.f;
                v.w = col + 3 < d ? src[3] : 0.f;
                *reinterpret_cast<float4*>(dst + lane * 4) = v;
            }
        }
    };

    if (wave < kProducers) {
        // ------------------------------------------------ producer
        const int li = lane & 15, lh = lane >> 4;
        const int qg = wave / DG, dg = wave % DG;
        // A operand: lane (i, h) holds query i's components 16*s + 4*h + e.
        float4 areg[QPB][S4];
#pragma unroll
        for (int qb = 0; qb < QPB; ++qb) {
            const int64_t q = q0 + (qg * QPB + qb) * 16 + li;
            const bool ok = q < nq;
            const float* row = xq + (ok ? q : 0) * d;
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4) areg[qb][s4] = load4_guard(row, 16 * s4 + 4 * lh, d, VEC, ok);
        }
        if (nsteps > 0) load_tile(c0, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int64_t s = 0; s <= nsteps; ++s) {
            if (s < nsteps) {
                if (s + 1 < nsteps) load_tile(c0 + (s + 1) * BN, (int)((s + 1) & 1));
                const float* bt = btile[s & 1];
                floatx4 acc[QPB][DPB];
#pragma unroll
                for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                    for (int db = 0; db < DPB; ++db) acc[qb][db] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s4 = 0; s4 < S4; ++s4) {
                    float4 b[DPB];
#pragma unroll
                    for (int db = 0; db < DPB; ++db) {
                        const int j = (dg * DPB + db) * 16 + li;
                        const int c = (4 * s4 + lh) ^ (j & SW);
                        b[db] = *reinterpret_cast<const float4*>(bt + (j * GR + c) * 4);
                    }
#pragma unroll
                    for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                        for (int db = 0; db < DPB; ++db) {
                            acc[qb][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[qb][s4].x, b[db].x, acc[qb][db], 0, 0, 0);
                            acc[qb][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[qb][s4].y, b[db].y, acc[qb][db], 0, 0, 0);
                            acc[qb][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[qb][s4].z, b[db].z, acc[qb][db], 0, 0, 0);
                            acc[qb][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[qb][s4].w, b[db].w, acc[qb][db], 0, 0, 0);
                        }
                }
                // D[i][j] of a 16x16 block sits in lane j + 16*(i/4), element i%4.
                float* slot = scores[s & 1];
#pragma unroll
                for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                    for (int db = 0; db < DPB; ++db)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            slot[((qg * QPB + qb) * 16 + 4 * lh + r) * LDP + (dg * DPB + db) * 16 + li] =
                                acc[qb][db][r];
                __builtin_amdgcn_s_waitcnt(0);
            }
            __syncthreads();
        }
    } else {
        // ------------------------------------------------ consumer
        // score = ||y||^2 - 2 q.y (L2) or -q.y (inner product); ||x||^2 is the
        // same for every candidate of a query and does not change its rank.
        const int cw = wave - kProducers;
        MultiSelect<KR, T, QW> sel;
        sel.init(keff);
        __syncthreads();
        float ynext = 0.f;
        if (L2 && c0 + lane < c1) ynext = yn[c0 + lane];
        for (int64_t s = 0; s <= nsteps; ++s) {
            if (s >= 1) {
                const float* slot = scores[(s - 1) & 1];
                const int64_t g = c0 + (s - 1) * BN + lane;
                const bool ok = g < c1;
                const float ynv = ynext;
                if (L2 && g + BN < c1) ynext = yn[g + BN];
                float score[QW];
#pragma unroll
                for (int qq = 0; qq < QW; ++qq) {
                    const float c = slot[(cw * QW + qq) * LDP + lane];
                    score[qq] = L2 ? fmaf(-2.f, c, ynv) : -c;
                }
                sel.offer(score, (uint32_t)g, ok);
            }
            __syncthreads();
        }
        sel.finish();
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) {
            const int64_t q = q0 + cw * QW + qq;
            if (q < nq) {
                uint64_t* out = part + (q * nchunks + chunk) * KS;
#pragma unroll
                for (int r = 0; r < KR; ++r) out[r * 64 + lane] = sel.w[qq][r];
            }
        }
    }
}

// Second pass: merge the chunks' partial lists of one query, recompute the
// kept candidates' distances in the direct form, re-rank, write k results.
constexpr int kMergeWaves = 4;
constexpr int kMaxDim = 512;

template <int KR>
__global__ __launch_bounds__(64 * kMergeWaves) void knn_merge_rerank(
    const uint64_t* __restrict__ part, int32_t nchunks, const float* __restrict__ xq, int64_t nq,
    const float* __restrict__ xb, int32_t d, int32_t vec, int32_t l2, int32_t k, int32_t keff,
    float* __restrict__ D, int64_t* __restrict__ I) {
    constexpr int T = SelParams<KR>::T;
    constexpr int KS = 64 * KR;
    __shared__ __align__(16) float xs[kMergeWaves][kMaxDim];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kMergeWaves + wave;
    if (q >= nq) return;

    WaveSelect<KR, T> ws;
    ws.init(keff);
    const uint64_t* p = part + q * nchunks * KS;
    // Each chunk's list is sorted; only its first keff entries can survive.
    const int per = (keff + 63) & ~63;
#pragma unroll 1
    for (int c = 0; c < nchunks; ++c) {
#pragma unroll 1
        for (int e = 0; e < per; e += 64) {
            const int i = e + lane;
            if (ws.push(i < keff ? p[(int64_t)c * KS + i] : kSentinel)) ws.merge();
        }
    }
    ws.finish();

    const float* x = xq + q * d;
    for (int t = lane; t < d; t += 64) xs[wave][t] = x[t];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");

    uint64_t nk[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const uint64_t key = ws.w[r];
        const int e = r * 64 + lane;
        nk[r] = kSentinel;
        if (key != kSentinel && e < keff) {
            const uint32_t i = key_index(key);
            const float* y = xb + (int64_t)i * d;
            float s = 0.f;
            if (vec) {
                for (int t = 0; t < d; t += 4) {
                    const float4 yv = *reinterpret_cast<const float4*>(y + t);
                    const float4 xv = *reinterpret_cast<const float4*>(&xs[wave][t]);
                    if (l2) {
                        float a = xv.x - yv.x, b = xv.y - yv.y, c = xv.z - yv.z, dd = xv.w - yv.w;
                        s = fmaf(a, a, s);
                        s = fmaf(b, b, s);
                        s = fmaf(c, c, s);
                        s = fmaf(dd, dd, s);
                    } else {
                        s = fmaf(xv.x, yv.x, s);
                        s = fmaf(xv.y, yv.y, s);
                        s = fmaf(xv.z, yv.z, s);
                        s = fmaf(xv.w, yv.w, s);
                    }
                }
            } else {
                for (int t = 0; t < d; ++t) {
                    if (l2) {
                        const float a = xs[wave][t] - y[t];
                        s = fmaf(a, a, s);
                    } else {
                        s = fmaf(xs[wave][t], y[t], s);
                    }
                }
            }
            nk[r] = make_key(l2 ? s : -s, i);
        }
    }
    bitonic_sort<false, KR>(nk);
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        if (e < k) {
            const uint64_t key = nk[r];
            if (key == kSentinel) {
                D[q * k + e] = l2 ? INFINITY : -INFINITY;
                I[q * k + e] = -1;
            } else {
                const float s = key_score(key);
                D[q * k + e] = l2 ? s : -s;
                I[q * k + e] = (int64_t)key_index(key);
            }
        }
    }
}

template <int KR, int DP>
mk_status knn_launch(const float* xq, int64_t nq, const float* xb, const float* yn, int64_t nb,
                     int32_t d, int32_t k, bool l2, bool vec, float* D, int64_t* I,
                     hipStream_t stream) {
    constexpr int BQ = FusedShape<KR, DP>::BQ;
    constexpr int BN = FusedShape<KR, DP>::BN;
    constexpr int KS = 64 * KR;
    const int keff = k + kSlack < KS ? k + kSlack : KS;
    const int64_t nqb = ceil_div(nq, BQ);
    // Chunks: enough workgroups to fill the chip several times over, but
    // long enough (>= 32 queue lengths) that partial lists stay small.
    int64_t want = ceil_div(4096, nqb);
    int64_t max_by_len = nb / (32 * KS) > 1 ? nb / (32 * KS) : 1;
    int64_t nchunks = want < max_by_len ? want : max_by_len;
    if (nchunks < 1) nchunks = 1;
    int64_t chunk_len = ceil_div(ceil_div(nb, nchunks), BN) * BN;
    if (chunk_len == 0) chunk_len = BN;
    nchunks = nb > 0 ? ceil_div(nb, chunk_len) : 1;

    Scratch part;
    mk_status st = part.alloc(sizeof(uint64_t) * (size_t)nq * (size_t)nchunks * KS, stream);
    if (st != MK_OK) return st;
    const int64_t nblocks = nqb * nchunks;
    MK_REQUIRE(nblocks < (1ll << 31), MK_ERR_UNSUPPORTED, "problem too large for one launch");
    {
        ProfScope prof("knn_fused", stream);
        auto kern = vec ? (l2 ? knn_fused<KR, DP, true, true> : knn_fused<KR, DP, true, false>)
                        : (l2 ? knn_fused<KR, DP, false, true> : knn_fused<KR, DP, false, false>);
        hipLaunchKernelGGL(kern, dim3((unsigned)nblocks),
                           dim3(64 * (kProducers + FusedShape<KR, DP>::NC)), 0, stream, xq, nq,
                           xb, yn, nb, d, chunk_len,
                           (int32_t)nchunks, (int32_t)nqb, keff, part.as<uint64_t>());
        MK_LAUNCHED();
    }
    {
        ProfScope prof("knn_merge_rerank", stream);
        hipLaunchKernelGGL((knn_merge_rerank<KR>), dim3((unsigned)ceil_div(nq, kMergeWaves)),
                           dim3(64 * kMergeWaves), 0, stream, part.as<uint64_t>(),
                           (int32_t)nchunks, xq, nq, xb, d, (int32_t)vec, (int32_t)l2, k, keff, D,
                           I);
        MK_LAUNCHED();
    }
    return MK_OK;
}

template <int DP>
mk_status knn_dispatch_k(const float* xq, int64_t nq, const float* xb, const float* yn,
                         int64_t nb, int32_t d, int32_t k, bool l2, bool vec, float* D, int64_t* I,
                         hipStream_t s) {
    const int want = k + kSlack < kMaxK ? k + kSlack : kMaxK;
    switch (queue_regs(want)) {
        case 1: return knn_launch<1, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
        case 2: return knn_launch<2, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
        case 4: return knn_launch<4, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
        case 8: return knn_launch<8, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
        default: return knn_launch<16, DP>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
    }
}

mk_status knn_search(const float* xq, int64_t nq, const float* xb, const float* yn_in, int64_t nb,
                     int32_t d, int32_t k, mk_metric metric, float* D, int64_t* I,
                     hipStream_t s) {
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
        mk_status st = norms.alloc(sizeof(float) * (size_t)nb, s);
        if (st != MK_OK) return st;
        st = launch_norms(xb, nb, d, norms.as<float>(), s);
        if (st != MK_OK) return st;
        yn = norms.as<float>();
    }
    if (d <= 32) return knn_dispatch_k<32>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
    if (d <= 64) return knn_dispatch_k<64>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
    if (d <= 96) return knn_dispatch_k<96>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
    if (d <= 128) return knn_dispatch_k<128>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
    return knn_dispatch_k<256>(xq, nq, xb, yn, nb, d, k, l2, vec, D, I, s);
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
