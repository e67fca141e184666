// Fused exact-search kernel shared by the FP32, BF16 and FP8 paths: MFMA
// distance tiles computed by producer waves feed register-resident selectors
// in consumer waves through LDS (Section 5.1 layout with the k-selection of
// Section 4.2 fused into the distance kernel), plus the second-pass merge and
// direct-form FP32 re-rank of the kept candidates.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "kselect.hpp"
#include "profile.hpp"
#include "wave_select.hpp"

namespace mk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// ---------------------------------------------------------------- selectors
// Chunks of one query tell each other how good their candidates are.  A
// chunk that holds r candidates scoring at most v proves that r rows of the
// database do; rows of different chunks are distinct, so once the proofs of
// all chunks add up to keff rows scoring at most t, no candidate scoring
// above t can enter the query's result.  Each chunk publishes four such
// points (v at ranks r0, 2 r0, 4 r0 and keff of its queue, r0 = ceil(keff /
// nchunks)); the tightest t that the published points prove is the query's
// bound, which is near the keff-th score of everything its chunks have seen
// so far, not merely of the best single chunk.
constexpr int kRankPoints = 4;
constexpr int kMaxRankChunks = 16;  // chunks per query when queues live in memory
constexpr uint32_t kNoBound = 0xFFFFFFFFu;

// QW independent selectors held by one wave (one per query the wave owns).
// Each queue register r (and each thread-queue slot) is a vector over the QW
// queries, low and high key halves apart, so that a merge can fetch and
// store the state of one query chosen at run time with a wave-uniform index
// (register-relative moves) instead of a select over all of them; the merge
// network is emitted once, not once per query.  A merge publishes the
// queue's rank points (above).  Queries at or beyond nvalid never take
// candidates.
template <int KR, int T, int QW>
struct MultiSelect {
    static constexpr int kQueries = QW;
    typedef uint32_t vq __attribute__((ext_vector_type(QW)));
    typedef float vqf __attribute__((ext_vector_type(QW)));
    vq wl[KR], wh[KR];   // wave queues
    vq tl[T], th[T];     // thread queues
    vq kl, kh;           // admission threshold key of each query (wave-uniform)
    vqf kf;              // its score
    vq bdu;              // order-mapped score bound from the chunks' rank points
    int cnt[QW];         // keys in each query's thread-queue buffer
    uint32_t* rpub;      // rank points of query q, this chunk, at rpub + q * rstride
    int64_t rstride;
    int rank[kRankPoints];
    int keff, nvalid;

    __device__ __forceinline__ void init(int k_eff, int valid, uint32_t* rank_base, int nchunks) {
        keff = k_eff;
        nvalid = valid;
        rpub = rank_base;
        rstride = (int64_t)nchunks * kRankPoints;
        const int r0 = (k_eff + nchunks - 1) / nchunks;
        rank[0] = r0;
        rank[1] = 2 * r0 < k_eff ? 2 * r0 : k_eff;
        rank[2] = 4 * r0 < k_eff ? 4 * r0 : k_eff;
        rank[3] = k_eff;
#pragma unroll
        for (int r = 0; r < KR; ++r) wl[r] = wh[r] = ~0u;
#pragma unroll
        for (int i = 0; i < T; ++i) tl[i] = th[i] = ~0u;
        kl = kh = ~0u;
        kf = INFINITY;
        bdu = kNoBound;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            cnt[q] = 0;
            if (q >= valid) {  // never admits a candidate
                kf[q] = -INFINITY;
                kl[q] = kh[q] = 0u;
            }
        }
    }

    // Lower query q's admission threshold to kk or the bound, whichever is
    // smaller; a candidate scoring exactly the bound still competes.
    __device__ __forceinline__ void set_threshold(int q, uint64_t kk) {
        const uint64_t bk = ((uint64_t)bdu[q] << 32) | 0xFFFFFFFFull;
        const uint64_t cur = ((uint64_t)kh[q] << 32) | kl[q];
        uint64_t th_key = kk < bk ? kk : bk;
        th_key = th_key < cur ? th_key : cur;
        kl[q] = (uint32_t)th_key;
        kh[q] = (uint32_t)(th_key >> 32);
        const uint32_t hi = (uint32_t)(th_key >> 32);
        kf[q] = fminf(kf[q], hi == kNoBound ? INFINITY : order_float(hi));
    }

    __device__ __forceinline__ void bound_u(int q, uint32_t b) {
        if (b < bdu[q]) {
            bdu[q] = b;
            set_threshold(q, ((uint64_t)kh[q] << 32) | kl[q]);
        }
    }

    __device__ __forceinline__ uint64_t key(int q, int r) const {
        return ((uint64_t)wh[r][q] << 32) | wl[r][q];
    }

    // Merge the thread queues of query q (wave-uniform) into its wave queue.
    __device__ __forceinline__ void merge_slot(int q) {
        uint64_t ww[KR], tt[T];
#pragma unroll
        for (int r = 0; r < KR; ++r) ww[r] = ((uint64_t)wh[r][q] << 32) | wl[r][q];
#pragma unroll
        for (int i = 0; i < T; ++i) tt[i] = ((uint64_t)th[i][q] << 32) | tl[i][q];
        ws_merge<KR, T>(ww, tt);
        const uint64_t kk = ws_element<KR>(ww, keff - 1);
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            wl[r][q] = (uint32_t)ww[r];
            wh[r][q] = (uint32_t)(ww[r] >> 32);
        }
#pragma unroll
        for (int i = 0; i < T; ++i) {
            tl[i][q] = ~0u;
            th[i][q] = ~0u;
        }
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) cnt[qq] = qq == q ? 0 : cnt[qq];
        set_threshold(q, kk);
        if (rpub && q < nvalid) {
            // the queue is sorted: its entry at rank r scores at most the
            // published value, as do the r - 1 before it
            const uint32_t p0 = (uint32_t)(ws_element<KR>(ww, rank[0] - 1) >> 32);
            const uint32_t p1 = (uint32_t)(ws_element<KR>(ww, rank[1] - 1) >> 32);
            const uint32_t p2 = (uint32_t)(ws_element<KR>(ww, rank[2] - 1) >> 32);
            if (lane_id() == 0) {
                uint64_t* rp = reinterpret_cast<uint64_t*>(rpub + (int64_t)q * rstride);
                __hip_atomic_store(rp, ((uint64_t)p1 << 32) | p0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(rp + 1, ((uint64_t)(uint32_t)(kk >> 32) << 32) | p2,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }

    // Offer, for every query q, this lane's candidate (score[q], idx); ok
    // false means no candidate.  A query whose scores all lose to its current
    // threshold is skipped after one compare per lane.
    __device__ __forceinline__ void offer(const float (&score)[QW], uint32_t idx, bool ok) {
        // one compare per query straight into a wave mask, one test of
        // their union with the lanes in range: the common case (no query
        // takes anything) costs two vector and one scalar instruction per
        // query and no per-query branch
        const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
        uint64_t cand[QW], any = 0;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            cand[q] = __builtin_amdgcn_ballot_w64(score[q] <= kf[q]);
            any |= cand[q];
        }
        if (!(any & okm)) return;
        uint32_t full = 0;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            if (cand[q] & okm) {
                const uint64_t key = ok ? make_key(score[q], idx) : kSentinel;
                const uint64_t kth = ((uint64_t)kh[q] << 32) | kl[q];
                const bool take = key < kth;
                const uint64_t bal = __ballot(take);
                if (bal) {
                    uint64_t tq[T];
#pragma unroll
                    for (int i = 0; i < T; ++i) tq[i] = ((uint64_t)th[i][q] << 32) | tl[i][q];
                    cnt[q] = tq_append<T>(tq, key, take, bal, cnt[q]);
#pragma unroll
                    for (int i = 0; i < T; ++i) {
                        tl[i][q] = (uint32_t)tq[i];
                        th[i][q] = (uint32_t)(tq[i] >> 32);
                    }
                    if (cnt[q] > 64 * (T - 1)) full |= 1u << q;
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
        for (int q = 0; q < nvalid; ++q) merge_slot(q);
    }
};

// s_waitcnt immediate (gfx9 encoding) that waits for all LDS operations.
constexpr int waitcnt_lgkm0() { return 0xF | (0x7 << 4) | (0x0 << 8) | (0x3 << 14); }

// Wave-wide reductions and scans over all 64 lanes.
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
    v = umin64(v, xor_lane64<1>(v));
    v = umin64(v, xor_lane64<2>(v));
    v = umin64(v, xor_lane64<4>(v));
    v = umin64(v, xor_lane64<8>(v));
    v = umin64(v, xor_lane64<16>(v));
    return umin64(v, xor_lane64<32>(v));
}
__device__ __forceinline__ uint64_t wave_max64(uint64_t v) {
    v = umax64(v, xor_lane64<1>(v));
    v = umax64(v, xor_lane64<2>(v));
    v = umax64(v, xor_lane64<4>(v));
    v = umax64(v, xor_lane64<8>(v));
    v = umax64(v, xor_lane64<16>(v));
    return umax64(v, xor_lane64<32>(v));
}
// Inclusive prefix sum over the wave's 64 lanes with DPP moves (no LDS
// round trip): shifts by 1, 2, 4 and 8 lanes inside each 16-lane row, then
// lane 15 of rows 0 and 2 added to rows 1 and 3 and lane 31 to rows 2 and 3.
// A lane whose source lies outside its row, or whose row is masked off,
// adds 0.
__device__ __forceinline__ int wave_inclusive_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// QW selectors for queues of 256 entries and more, whose candidates live in
// device memory -- the kernel's own partial-result rows.  A candidate that
// beats its query's threshold is appended to the query's pool (one store per
// wave, positions from the ballot); nothing is kept sorted while the chunk
// is scanned.  When a pool nears its capacity (twice the queue) it is cut
// back to about keff keys by a radix selection over the 64-bit keys: a
// histogram of NB bins over [smallest, largest] key, built with LDS atomics,
// locates the bin holding the keff-th smallest key, and the search recurses
// into that bin until at most `target` keys remain at or below its upper
// edge.  The kept keys are the smallest ones (bins are monotone in the key),
// at least keff of them, and the largest kept key + 1 becomes the threshold:
// a key above it cannot be among the keff smallest.  A selection costs a few
// passes over 2*64*KR keys for about 64*KR insertions, where a sorted queue
// pays a full merge network every 64-128.  At the end the pool is cut to at
// most 64*KR keys and padded with sentinels; the second pass selects from
// it.  The level-0 histogram also yields the rank points published for the
// other chunks (see above).  Queries at or beyond nvalid never take
// candidates and are never written.
template <int KR, int QW, int NB, int RB = 16>
struct PoolSelect {
    static constexpr int kQueries = QW;
    static constexpr int KS = 64 * KR;
    static constexpr int CAP = 2 * KS;  // pool capacity in keys
    static constexpr int PRG = CAP / 64;
    static constexpr int kRB = PRG < RB ? PRG : RB;  // pool rows per lane loaded together
    static constexpr int NBL = NB / 64;  // bins per lane in a scan
    static constexpr int LOGNB = NB == 1024 ? 10 : NB == 512 ? 9 : NB == 256 ? 8 : 7;
    static_assert(NB == 1024 || NB == 512 || NB == 256 || NB == 128, "bins");
    typedef uint32_t vq __attribute__((ext_vector_type(QW)));
    typedef float vqf __attribute__((ext_vector_type(QW)));
    vq kl, kh;           // admission threshold key of each query (wave-uniform)
    vqf kf;              // its score
    vq bdu;              // order-mapped score bound from the chunks' rank points
    int cnt[QW];         // keys in each query's pool
    // set when an append takes some pool past the refine level / the
    // urgency level, so that the per-step checks cost one scalar test
    bool need_cut, is_urgent;
    uint64_t* wbase;     // pool of query q at wbase + q * wstride
    int64_t wstride;
    uint32_t* rpub;      // rank points of query q, this chunk, at rpub + q * rstride
    int64_t rstride;
    uint32_t* hist;      // NB zeroed counters in LDS, private to this wave
    unsigned long long* drops;  // keys an overfull pool could not hold (stays 0)
    int rank[kRankPoints];
    int keff, nvalid;

    __device__ __forceinline__ void init(int k_eff, uint64_t* base, int64_t stride, int valid,
                                         uint32_t* rank_base, int nchunks, uint32_t* bins,
                                         unsigned long long* drop_count) {
        keff = k_eff;
        drops = drop_count;
        wbase = base;
        wstride = stride;
        nvalid = valid;
        rpub = rank_base;
        rstride = (int64_t)nchunks * kRankPoints;
        hist = bins;
        const int r0 = (k_eff + nchunks - 1) / nchunks;
        rank[0] = r0;
        rank[1] = 2 * r0 < k_eff ? 2 * r0 : k_eff;
        rank[2] = 4 * r0 < k_eff ? 4 * r0 : k_eff;
        rank[3] = k_eff;
        kl = kh = ~0u;
        kf = INFINITY;
        bdu = kNoBound;
        need_cut = is_urgent = false;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            cnt[q] = 0;
            if (q >= valid) {  // never admits a candidate
                kf[q] = -INFINITY;
                kl[q] = kh[q] = 0u;
            }
        }
        const int lane = lane_id();
#pragma unroll
        for (int j = 0; j < NBL; ++j) hist[lane * NBL + j] = 0u;
    }

    // Lower query q's admission threshold to kk or the bound, whichever is
    // smaller; a candidate scoring exactly the bound still competes (its key
    // is below the bound's key for any index).
    __device__ __forceinline__ void set_threshold(int q, uint64_t kk) {
        const uint64_t bk = ((uint64_t)bdu[q] << 32) | 0xFFFFFFFFull;
        const uint64_t cur = ((uint64_t)kh[q] << 32) | kl[q];
        uint64_t th_key = kk < bk ? kk : bk;
        th_key = th_key < cur ? th_key : cur;
        kl[q] = (uint32_t)th_key;
        kh[q] = (uint32_t)(th_key >> 32);
        const uint32_t hi = (uint32_t)(th_key >> 32);
        kf[q] = fminf(kf[q], hi == kNoBound ? INFINITY : order_float(hi));
    }

    __device__ __forceinline__ void bound_u(int q, uint32_t b) {
        if (b < bdu[q]) {
            bdu[q] = b;
            set_threshold(q, ((uint64_t)kh[q] << 32) | kl[q]);
        }
    }

    // Position of the t-th smallest key (1-based) in the histogram whose
    // lane-local bins are h and lane-exclusive prefix excl (wave totals
    // incl): its bin, and the keys in the bins before it and up to it.
    // False when the histogram holds fewer than t keys.
    __device__ __forceinline__ bool locate(const uint32_t (&h)[NBL], int excl, int incl, int t,
                                           int& bin, int& before, int& upto) const {
        int jl = NBL - 1, cb = incl, ci = incl, c = excl;
        bool f = false;
#pragma unroll
        for (int j = 0; j < NBL; ++j) {
            const int c2 = c + (int)h[j];
            if (!f && c2 >= t) {
                jl = j;
                cb = c;
                ci = c2;
                f = true;
            }
            c = c2;
        }
        const uint64_t m = __ballot(excl < t && t <= incl);
        if (!m) return false;
        const int L = __builtin_ctzll(m);
        bin = L * NBL + __builtin_amdgcn_readlane(jl, L);
        before = __builtin_amdgcn_readlane(cb, L);
        upto = __builtin_amdgcn_readlane(ci, L);
        return true;
    }

    // Cut query q's pool to the keys at or below a bin edge such that at
    // least keff and at most `target` keys remain (all of them when it
    // holds no more than target), refresh its threshold and publish its
    // rank points.
    __device__ __forceinline__ void refine(int q, int target) {
        const int lane = lane_id();
        uint64_t* pp = wbase + (int64_t)q * wstride;
        int n = 0;
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) n = qq == q ? cnt[qq] : n;
        if (n <= target) return;
        // the appends of every lane of this wave are visible to its loads
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        // Each pass loads the pool in batches of kRB rows per lane, issued
        // together (indices clamped into the pool, so no load is guarded):
        // a cut's latency is a few round trips, not one per row.
        auto batch = [&](int r0, uint64_t (&kk)[kRB]) __attribute__((always_inline)) {
#pragma unroll
            for (int b = 0; b < kRB; ++b) {
                const int i = (r0 + b) * 64 + lane;
                kk[b] = pp[i < n ? i : n - 1];
            }
        };
        uint64_t lo = kSentinel, hi = 0;
#pragma unroll 1
        for (int r0 = 0; r0 * 64 < n; r0 += kRB) {
            uint64_t kk[kRB];
            batch(r0, kk);
#pragma unroll
            for (int b = 0; b < kRB; ++b) {
                lo = umin64(lo, kk[b]);
                hi = umax64(hi, kk[b]);
            }
        }
        lo = wave_min64(lo);
        hi = wave_max64(hi);
        uint32_t pts[3] = {kNoBound, kNoBound, kNoBound};
        uint64_t cut = hi;
        int below = 0;
#pragma unroll 1
        for (int level = 0; level < 10; ++level) {
            const uint64_t range = hi - lo;
            const int bits = range ? 64 - __builtin_clzll(range) : 0;
            const int shift = bits > LOGNB ? bits - LOGNB : 0;
#pragma unroll 1
            for (int r0 = 0; r0 * 64 < n; r0 += kRB) {
                uint64_t kk[kRB];
                batch(r0, kk);
#pragma unroll
                for (int b = 0; b < kRB; ++b) {
                    const uint64_t k = kk[b];
                    if ((r0 + b) * 64 + lane < n && k >= lo && k <= hi)
                        atomicAdd(&hist[(uint32_t)((k - lo) >> shift)], 1u);
                }
            }
            __builtin_amdgcn_s_waitcnt(waitcnt_lgkm0());
            uint32_t h[NBL];
            int tot = 0;
#pragma unroll
            for (int j = 0; j < NBL; ++j) {
                h[j] = hist[lane * NBL + j];
                tot += (int)h[j];
            }
#pragma unroll
            for (int j = 0; j < NBL; ++j) hist[lane * NBL + j] = 0u;
            const int incl = wave_inclusive_sum(tot);
            const int excl = incl - tot;
            // upper edge key of bin b, clamped to hi
            auto edge = [&](int b) -> uint64_t {
                const uint64_t off = ((uint64_t)(b + 1) << shift) - 1;
                return off >= range ? hi : lo + off;
            };
            if (level == 0) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    int b, bf, up;
                    if (locate(h, excl, incl, rank[j], b, bf, up)) pts[j] = (uint32_t)(edge(b) >> 32);
                }
            }
            int b, bf, up;
            if (!locate(h, excl, incl, keff - below, b, bf, up)) break;  // cannot happen: n > keff
            if (below + up <= target || shift == 0) {
                cut = edge(b);
                break;
            }
            below += bf;
            const uint64_t nhi = edge(b);
            lo = lo + ((uint64_t)b << shift);
            hi = nhi;
        }
        // keep the keys at or below the cut, packed at the front
        // (in place: a batch's stores land at or below its own rows, after
        // its loads, and below every row of the later batches)
        int kept = 0;
        uint64_t top = 0;
#pragma unroll 1
        for (int r0 = 0; r0 * 64 < n; r0 += kRB) {
            uint64_t kk[kRB];
            batch(r0, kk);
#pragma unroll
            for (int b = 0; b < kRB; ++b) {
                const uint64_t k = kk[b];
                const bool keep = (r0 + b) * 64 + lane < n && k <= cut;
                const uint64_t bal = __ballot(keep);
                const int pos = kept + (int)__builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(bal >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (keep) pp[pos] = k;
                top = keep ? umax64(top, k) : top;
                kept += __popcll(bal);
            }
        }
        top = wave_max64(top);
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) cnt[qq] = qq == q ? kept : cnt[qq];
        set_threshold(q, top + 1);
        if (rpub && lane == 0) {
            uint64_t* rp = reinterpret_cast<uint64_t*>(rpub + (int64_t)q * rstride);
            __hip_atomic_store(rp, ((uint64_t)pts[1] << 32) | pts[0], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(rp + 1, ((uint64_t)(uint32_t)(top >> 32) << 32) | pts[2],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    __device__ __forceinline__ void offer(const float (&score)[QW], uint32_t idx, bool ok) {
        uint32_t full = 0;
        const int lane = lane_id();
        // one compare per query straight into a wave mask, one test of
        // their union with the lanes in range
        const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
        uint64_t cand[QW], any = 0;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            cand[q] = __builtin_amdgcn_ballot_w64(score[q] <= kf[q]);
            any |= cand[q];
        }
        if (!(any & okm)) return;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            if (cand[q] & okm) {
                const uint64_t key = ok ? make_key(score[q], idx) : kSentinel;
                const uint64_t kth = ((uint64_t)kh[q] << 32) | kl[q];
                const bool take = key < kth;
                const uint64_t bal = __ballot(take);
                if (bal) {
                    const int below = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                    if (take) {
                        if (cnt[q] + below < CAP)
                            wbase[(int64_t)q * wstride + cnt[q] + below] = key;
                        else if (drops)  // refine_pools() runs first: never taken
                            atomicAdd(drops, 1ull);
                    }
                    cnt[q] += __popcll(bal);
                    need_cut |= cnt[q] > CAP - 64;
                    is_urgent |= kBatch && cnt[q] > kUrgent;
                }
            }
        }
        (void)lane;
        (void)full;
    }

    // Long selections (pools of 2048 keys) are batched across the consumers
    // of a workgroup: one wave's selection stalls every wave at the next
    // barrier, so when any consumer has a pool within three offers of its
    // capacity (`urgent`), all of them cut every pool that is at least half
    // way from keff to capacity in the same step.  A pool that could
    // overflow in the next offer is cut anyway.
    static constexpr bool kBatch = CAP >= 2048;
    static constexpr int kUrgent = CAP - 192;
    __device__ __forceinline__ bool urgent() const { return kBatch && is_urgent; }
    __device__ __forceinline__ void refine_pools(bool batch) {
        if (!batch && !need_cut) return;  // no pool can overflow in the next offer
        const int level = batch ? (keff + CAP) / 2 : CAP - 64;
        uint32_t m = 0;
#pragma unroll
        for (int q = 0; q < QW; ++q) m |= (cnt[q] > level ? 1u : 0u) << q;
        while (m) {
            const int q = __builtin_ctz(m);
            m &= m - 1;
            refine(q, keff + 128);
        }
        // every pool above `level` was cut to at most keff + 128 keys
        need_cut = false;
        bool u = false;
#pragma unroll
        for (int q = 0; q < QW; ++q) u |= cnt[q] > kUrgent;
        is_urgent = kBatch && u;
    }

    // Cut every valid query's pool to at most 64*KR keys and pad it with
    // sentinels to that length: the chunk's unsorted candidate list.
    __device__ __forceinline__ void finish() {
        const int lane = lane_id();
#pragma unroll 1
        for (int q = 0; q < nvalid; ++q) {
            refine(q, KS);
            int n = 0;
#pragma unroll
            for (int qq = 0; qq < QW; ++qq) n = qq == q ? cnt[qq] : n;
            uint64_t* pp = wbase + (int64_t)q * wstride;
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                const int i = r * 64 + lane;
                if (i >= n) pp[i] = kSentinel;
            }
        }
    }

};

// Tighten every query's bound from the rank points all chunks have
// published (bound[q][c][0..3], at most kMaxRankChunks chunks): each chunk's
// points are proposed as bounds, the rows each proposal is proven for are
// counted over every chunk, and the smallest proposal proven for keff rows
// wins.  Here one lane per chunk serves a query, four queries per pass (few
// registers, for the register-queue selectors).
template <class Sel>
__device__ __forceinline__ void exchange_ranks(Sel& sel, const uint32_t* bound, int nchunks,
                                               int64_t qfirst, int64_t nq) {
    constexpr int QW = Sel::kQueries;
    constexpr int G = kMaxRankChunks;
    constexpr int QPP = 64 / G;
    static_assert(G * QPP == 64, "lanes per query");
    const int lane = lane_id();
    const int m = lane % G, sub = lane / G;
#pragma unroll 1
    for (int p = 0; p < (QW + QPP - 1) / QPP; ++p) {
        const int qq = p * QPP + sub;
        const int64_t q = qfirst + qq;
        const bool qok = qq < QW && q < nq;
        uint32_t cand[kRankPoints];
        uint64_t lo = ~0ull, hi = ~0ull;
        if (qok && m < nchunks) {
            const uint64_t* src = reinterpret_cast<const uint64_t*>(bound + q * sel.rstride) + 2 * m;
            lo = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            hi = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        cand[0] = (uint32_t)lo;
        cand[1] = (uint32_t)(lo >> 32);
        cand[2] = (uint32_t)hi;
        cand[3] = (uint32_t)(hi >> 32);
        int rows[kRankPoints] = {0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < G; ++c) {
            if (c < nchunks) {
                const int from = sub * G + c;
                uint32_t v[kRankPoints];
#pragma unroll
                for (int j = 0; j < kRankPoints; ++j) v[j] = (uint32_t)__shfl((int)cand[j], from);
#pragma unroll
                for (int j = 0; j < kRankPoints; ++j) {
                    const uint32_t t = cand[j];
                    rows[j] += v[3] <= t   ? sel.rank[3]
                               : v[2] <= t ? sel.rank[2]
                               : v[1] <= t ? sel.rank[1]
                               : v[0] <= t ? sel.rank[0]
                                           : 0;
                }
            }
        }
        uint32_t best = kNoBound;
#pragma unroll
        for (int j = 0; j < kRankPoints; ++j)
            if (rows[j] >= sel.keff && cand[j] < best) best = cand[j];
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const uint32_t other = (uint32_t)__shfl_xor((int)best, o);
            best = other < best ? other : best;
        }
#pragma unroll
        for (int j = 0; j < QW; ++j)
            if (j / QPP == p && qfirst + j < nq)
                sel.bound_u(j, (uint32_t)__builtin_amdgcn_readlane((int)best, (j % QPP) * G));
    }
}

// One pass for all QW queries, 64 / QW lanes per query (lane m proposes the
// points of chunks m, m + 64/QW, ...): fewer round trips, more registers.
template <class Sel>
__device__ __forceinline__ void exchange_ranks_wide(Sel& sel, const uint32_t* bound, int nchunks,
                                                    int64_t qfirst, int64_t nq) {
    constexpr int QW = Sel::kQueries;
    constexpr int G = 64 / QW;
    constexpr int CPL = kMaxRankChunks / G > 0 ? kMaxRankChunks / G : 1;
    static_assert(G * QW == 64, "one query per G lanes");
    const int lane = lane_id();
    const int qq = lane / G, m = lane % G;
    const int64_t q = qfirst + qq;
    const bool qok = q < nq;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(bound + (qok ? q : 0) * sel.rstride);
    uint32_t cand[CPL][kRankPoints];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = m + G * u;
        uint64_t lo = ~0ull, hi = ~0ull;
        if (qok && c < nchunks) {
            lo = __hip_atomic_load(src + 2 * c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            hi = __hip_atomic_load(src + 2 * c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        cand[u][0] = (uint32_t)lo;
        cand[u][1] = (uint32_t)(lo >> 32);
        cand[u][2] = (uint32_t)hi;
        cand[u][3] = (uint32_t)(hi >> 32);
    }
    int rows[CPL][kRankPoints];
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
        for (int j = 0; j < kRankPoints; ++j) rows[u][j] = 0;
    // chunk c's points are held by lane (qq * G + c % G), slot c / G
#pragma unroll
    for (int c = 0; c < kMaxRankChunks; ++c) {
        if (c < nchunks) {
            const int from = qq * G + c % G;
            uint32_t v[kRankPoints];
#pragma unroll
            for (int j = 0; j < kRankPoints; ++j)
                v[j] = (uint32_t)__shfl((int)cand[c / G][j], from);
#pragma unroll
            for (int u = 0; u < CPL; ++u) {
                if (G * u < nchunks) {
#pragma unroll
                    for (int j = 0; j < kRankPoints; ++j) {
                        const uint32_t t = cand[u][j];
                        rows[u][j] += v[3] <= t   ? sel.rank[3]
                                      : v[2] <= t ? sel.rank[2]
                                      : v[1] <= t ? sel.rank[1]
                                      : v[0] <= t ? sel.rank[0]
                                                  : 0;
                    }
                }
            }
        }
    }
    uint32_t best = kNoBound;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
        for (int j = 0; j < kRankPoints; ++j)
            if (rows[u][j] >= sel.keff && cand[u][j] < best) best = cand[u][j];
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const uint32_t other = (uint32_t)__shfl_xor((int)best, o);
        best = other < best ? other : best;
    }
#pragma unroll
    for (int j = 0; j < QW; ++j)
        if (qfirst + j < nq) sel.bound_u(j, (uint32_t)__builtin_amdgcn_readlane((int)best, j * G));
}

// ---------------------------------------------------------------- operands
// Operand formats of the distance tile.  A 16-byte granule holds EPG
// elements; lane (i, h) of a 16x16 MFMA block supplies granule 4*s + h of
// its query (A) or database row (B) at granule step s, so both operands use
// the same component order and the sum over components is exact-order
// independent of it.
struct OpF32 {   // v_mfma_f32_16x16x4f32, four per granule
    static constexpr int CONSUMERS = 4;
    static constexpr int EPG = 4;
    static constexpr int BYTES = 4;
    static constexpr bool SCALED = false;
    __device__ static __forceinline__ floatx4 mma(floatx4 c, uint4 a, uint4 b) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
        return c;
    }
};
// The low-precision tiles take the matrix cores a fraction of the FP32 time,
// so their workgroups run eight consumer waves to keep up (rows of up to 256
// bytes, whose producers fit the smaller register budget).
struct OpBF16 {  // v_mfma_f32_16x16x32_bf16, one per granule
    static constexpr int CONSUMERS = 8;
    static constexpr int EPG = 8;
    static constexpr int BYTES = 2;
    static constexpr bool SCALED = false;
    __device__ static __forceinline__ floatx4 mma(floatx4 c, uint4 a, uint4 b) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};
struct OpFP8 {   // v_mfma_f32_16x16x32_fp8_fp8 (OCP E4M3), two per granule
    static constexpr int CONSUMERS = 8;
    static constexpr int EPG = 16;
    static constexpr int BYTES = 1;
    static constexpr bool SCALED = true;
    __device__ static __forceinline__ floatx4 mma(floatx4 c, uint4 a, uint4 b) {
        const long a0 = (long)(((uint64_t)a.y << 32) | a.x), a1 = (long)(((uint64_t)a.w << 32) | a.z);
        const long b0 = (long)(((uint64_t)b.y << 32) | b.x), b1 = (long)(((uint64_t)b.w << 32) | b.z);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, c, 0, 0, 0);
        return c;
    }
};

// Granule c (16 bytes) of a row with `stride` elements of which the first
// `valid` are real; granules past `valid` read as zero.  Rows whose length in
// bytes is not a multiple of 16 take the element-wise path (FP32 only).
template <class Op, bool VEC>
__device__ __forceinline__ uint4 load_granule(const void* row_base, int c, int valid, bool ok) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (!ok) return v;
    const int e0 = c * Op::EPG;
    if constexpr (VEC) {
        if (e0 < valid)
            v = *reinterpret_cast<const uint4*>(static_cast<const unsigned char*>(row_base) + (size_t)e0 * Op::BYTES);
    } else {
        static_assert(Op::BYTES == 4, "element-wise path is FP32 only");
        const float* r = static_cast<const float*>(row_base);
        if (e0 < valid) v.x = __float_as_uint(r[e0]);
        if (e0 + 1 < valid) v.y = __float_as_uint(r[e0 + 1]);
        if (e0 + 2 < valid) v.z = __float_as_uint(r[e0 + 2]);
        if (e0 + 3 < valid) v.w = __float_as_uint(r[e0 + 3]);
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

// s_waitcnt immediate (gfx9 encoding) that waits until at most N vector
// memory operations are outstanding and for all LDS operations.
template <int N>
constexpr int waitcnt_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt is 6 bits");
    return (N & 0xF) | (0x7 << 4) | (0x0 << 8) | (((N >> 4) & 0x3) << 14);
}

// Workgroup of the fused kernel: 4 producer waves (one per SIMD) compute the
// q.y tile of BQ queries x BN = 64 database rows per step on the matrix
// cores and write it to one of two LDS slots, while NC consumer waves (4 for
// FP32, 8 for the low-precision formats) run the selectors of the previous
// step's tile from the other slot -- MFMA and VALU selection overlap, one
// barrier per step.  Each producer owns QPB query blocks x DPB database
// blocks of 16 (a 4-producer grid of QG x DG), each consumer QW = BQ/NC
// queries.  BQ = 64, or 16 for rows over 512 bytes (LDS).
constexpr int kProducers = 4;

// Queues of 256 entries and more live in device memory (GlobalSelect).
constexpr bool queues_in_memory(int KR) { return KR >= 4; }

template <class Op, int DP>
constexpr int fused_consumers() {
    return DP * Op::BYTES <= 256 ? Op::CONSUMERS : 4;
}

template <int KR, int RB, int NCONS = 4>
struct FusedShape {
    static constexpr bool mem_queues = queues_in_memory(KR);
    static constexpr int NC = NCONS;
    // waves per SIMD: the producers and consumers of one workgroup
    static constexpr int WPE = (kProducers + NC) / 4;
    // thread-queue buffer: 64*T keys per query
    static constexpr int T = SelParams<KR>::T;
    // keys of one (query, chunk) row of partial results: a sorted queue, or
    // a candidate pool of twice the queue length
    static constexpr int ROW = (mem_queues ? 2 : 1) * 64 * KR;
    static constexpr bool wide = RB > 512;
    static constexpr int QPB = wide ? 1 : 2;
    static constexpr int DPB = wide ? 1 : 2;
    static constexpr int DG = DPB == 2 ? 2 : 4;
    static constexpr int QG = kProducers / DG;
    static constexpr int BQ = QG * QPB * 16;
    static constexpr int BN = DG * DPB * 16;
    static constexpr int QW = BQ / NC;
    static_assert(BN == 64, "consumers take one column per lane");
};

// Per-call arguments of the fused kernel.
struct FusedArgs {
    const void* xq;       // queries, `stride` elements per row
    const void* xb;       // database rows, same format
    const float* yn;      // ||y||^2 per row (L2 only)
    const float* qinv;    // per-query 1/scale (scaled formats only)
    const float* yinv;    // per-row 1/scale (scaled formats only)
    int64_t nq, nb;
    int32_t stride;       // elements per row in memory
    int32_t valid;        // leading elements per row that are real (rest zero)
    int64_t chunk_len;
    int32_t nchunks, nqb, keff;
    uint64_t* part;       // [nq][nchunks][ROW] keys: each chunk's queue (and pool)
    // rank points shared by the chunks of a query, [nq][nchunks][4]
    uint32_t* bound;
    // debug count of candidates a full pool had to drop (must stay zero)
    unsigned long long* drops;
};

template <class Op, int KR, int DP, bool VEC, bool L2>
__global__ __launch_bounds__(64 * (kProducers + fused_consumers<Op, DP>())) __attribute__((
    amdgpu_waves_per_eu((kProducers + fused_consumers<Op, DP>()) / 4,
                        (kProducers + fused_consumers<Op, DP>()) / 4))) void
knn_fused(FusedArgs args) {
    using S = FusedShape<KR, DP * Op::BYTES, fused_consumers<Op, DP>()>;
    constexpr int T = S::T;
    constexpr int BQ = S::BQ, BN = S::BN, QW = S::QW, QPB = S::QPB, DPB = S::DPB, DG = S::DG;
    // Score slot: column-major, LDQ floats per database row (a multiple of 4,
    // 4 mod 32 words apart) so that producers store four queries of a column
    // and consumers load their QW queries of a column as 16-byte vectors
    // without bank conflicts.
    constexpr int LDQ = BQ + 4 + ((BQ + 4) % 32 == 4 ? 0 : (36 - (BQ + 4) % 32) % 32);
    static_assert(LDQ % 4 == 0 && QW % 2 == 0, "vector score access");
    constexpr int KS = 64 * KR;
    // Database tile in LDS: BN rows of GR 16-byte granules; granule c of row j
    // is stored at position c ^ (j & SW) so that the 16 rows read by one MFMA
    // operand load fall in different banks.
    constexpr int GR = DP / Op::EPG;
    constexpr int S4 = GR / 4;  // granule steps per row
    static_assert(GR % 4 == 0, "padded row must be a multiple of 4 granules");
    constexpr int SW = (GR % 16 == 0) ? 15 : (GR % 8 == 0) ? 7 : 3;
    constexpr int NI = BN * GR / 64;  // 64-lane granule loads per tile
    constexpr int SK0 = 4 / (QPB * DPB) > 1 ? 4 / (QPB * DPB) : 1;
    constexpr int SK = SK0 < S4 ? SK0 : S4;

    constexpr int LPW = NI / kProducers;  // tile loads per producer wave
    static_assert(NI % kProducers == 0, "tile loads split evenly over the producers");
    // Per-row side values of a tile (||y||^2 for L2, 1/scale for scaled
    // formats) travel to LDS with it: producer wave r < NSIDE loads side
    // array r for the tile's rows, one 4-byte load per lane, into a ring of
    // NBUF + 1 slots, so the consumers' step loop issues no global load and
    // never waits on the vector-memory counter, which on this chip also
    // counts their own pool stores.
    constexpr int NSIDE = (L2 ? 1 : 0) + (Op::SCALED ? 1 : 0);
    // Database tiles in flight: as many buffers as the LDS left after the
    // score slots and the smallest histograms holds (at most 6), loads
    // running NBUF - 1 steps ahead; the steps' barriers do not wait for
    // them, only each step's own tile is waited for (vmcnt counts up to 63
    // outstanding loads).
    constexpr int kLdsBytes = 160 * 1024;
    constexpr int TILE_BYTES = BN * GR * 16;
    constexpr int SIDE_BYTES = NSIDE * 7 * BN * 4;
    constexpr int OTHER = 2 * BN * LDQ * 4 + SIDE_BYTES + (S::mem_queues ? S::NC * 128 * 4 : 0) + 512;
    constexpr int NB_LDS = (kLdsBytes - OTHER) / TILE_BYTES;
    constexpr int NB_VM = 63 / (LPW + (NSIDE > 0 ? 1 : 0)) + 1;
    constexpr int NB0 = NB_LDS < NB_VM ? NB_LDS : NB_VM;
    constexpr int NBUF = NB0 > 6 ? 6 : NB0 < 2 ? 2 : NB0;
    constexpr int AHEAD = NBUF - 1;

    // one statically named array per buffer, so that loads into one buffer
    // and reads of another are told apart without waiting
    __shared__ __align__(16) uint4 bt0[BN * GR];
    __shared__ __align__(16) uint4 bt1[BN * GR];
    __shared__ __align__(16) uint4 bt2[NBUF > 2 ? BN * GR : 1];
    __shared__ __align__(16) uint4 bt3[NBUF > 3 ? BN * GR : 1];
    __shared__ __align__(16) uint4 bt4[NBUF > 4 ? BN * GR : 1];
    __shared__ __align__(16) uint4 bt5[NBUF > 5 ? BN * GR : 1];
    auto tile_buf = [&](int u) __attribute__((always_inline)) -> uint4* {
        return u == 0 ? bt0 : u == 1 ? bt1 : u == 2 ? bt2 : u == 3 ? bt3 : u == 4 ? bt4 : bt5;
    };
    // LDS byte address of buffer u (each array's own address, a constant,
    // so no generic-pointer conversion is left for the loads to pay)
    auto tile_lds = [&](int u) __attribute__((always_inline)) -> uint32_t {
        return u == 0   ? (uint32_t)(uintptr_t)(lds_ptr_t)bt0
               : u == 1 ? (uint32_t)(uintptr_t)(lds_ptr_t)bt1
               : u == 2 ? (uint32_t)(uintptr_t)(lds_ptr_t)bt2
               : u == 3 ? (uint32_t)(uintptr_t)(lds_ptr_t)bt3
               : u == 4 ? (uint32_t)(uintptr_t)(lds_ptr_t)bt4
                        : (uint32_t)(uintptr_t)(lds_ptr_t)bt5;
    };
    __shared__ __align__(16) float scores[2][BN * LDQ];
    __shared__ __align__(16) float side[NSIDE > 0 ? NSIDE : 1][NBUF + 1][BN];
    // histogram bins of each consumer's pool selections: as many as the LDS
    // left over allows (at most 1024)
    constexpr int USED = NBUF * BN * GR * 16 + 2 * BN * LDQ * 4 + SIDE_BYTES;
    constexpr int NBINS = !S::mem_queues                             ? 1
                          : USED + S::NC * 1024 * 4 <= kLdsBytes     ? 1024
                          : USED + S::NC * 512 * 4 <= kLdsBytes      ? 512
                          : USED + S::NC * 256 * 4 <= kLdsBytes      ? 256
                                                                     : 128;
    static_assert(!S::mem_queues || USED + S::NC * NBINS * 4 <= kLdsBytes, "LDS");
    __shared__ uint32_t bins[S::mem_queues ? S::NC : 1][NBINS];
    __shared__ uint32_t urgent_flags[2][S::NC];

    const int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)args.nqb * args.nchunks);
    const int64_t chunk = logical / args.nqb;
    const int64_t qblk = logical % args.nqb;
    // wave-uniform, and known to be so (scalar registers, scalar branches)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int64_t q0 = qblk * BQ;
    const int64_t c0 = chunk * args.chunk_len;
    const int64_t c1 = c0 + args.chunk_len < args.nb ? c0 + args.chunk_len : args.nb;
    // 32-bit step counters (scalar compares): a chunk has fewer than 2^31 rows
    const int nsteps = c1 > c0 ? (int)((c1 - c0 + BN - 1) / BN) : 0;
    const int64_t row_bytes = (int64_t)args.stride * Op::BYTES;
    const unsigned char* xb = static_cast<const unsigned char*>(args.xb);

    // Load the tile of rows [t0, t0 + BN) into btile[buf]; producers share
    // the NI granule loads, LPW per wave, whose per-lane byte offsets inside a
    // tile are fixed (loff).  Rows past the chunk repeat its last row and
    // granules past the valid elements repeat granule 0: both only ever meet
    // zero A components or unconsumed score columns.
    // (row j inside the tile, granule cc of the row) of load t of this lane;
    // only the fast path keeps its offsets, the others recompute them
    auto granule_of = [&](int t, int& j, int& cc) __attribute__((always_inline)) {
        const int g = (wave + t * kProducers) * 64 + lane;
        j = g / GR;
        const int c = (g % GR) ^ (j & SW);
        cc = c * Op::EPG < args.valid ? c : 0;
    };
    int32_t loff[LPW];
#pragma unroll
    for (int t = 0; t < LPW; ++t) {
        int j, cc;
        granule_of(t, j, cc);
        loff[t] = (int32_t)(j * row_bytes + cc * 16);
    }
    // Direct global-to-LDS load of 16 bytes per lane (lane i writes at LDS
    // byte address m0 + 16 i).  Issued from asm so that the compiler's wait
    // insertion does not see an LDS write in flight: it would otherwise wait
    // for every such load before any later LDS read or barrier fence.  It
    // writes no register; its completion is waited for by the explicit
    // vmcnt waits of the step loop (producers issue no other vector memory
    // operations there).  An LDS DMA load needs one wait state after the
    // write of M0 (the s_nop; the compiler inserts the same for its own such
    // loads).  M0 is reserved to the compiler, which sets it before each of
    // its own uses; the kernel's generated code has no M0 user but these
    // loads.
    auto dma16 = [&](const unsigned char* src, uint32_t m0) __attribute__((always_inline)) {
        asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                     :
                     : "v"(src), "s"(m0)
                     : "memory", "m0");
    };
    auto dma4 = [&](const float* src, uint32_t m0) __attribute__((always_inline)) {
        asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
                     :
                     : "v"(src), "s"(m0)
                     : "memory", "m0");
    };
    // side values of the tile at t0 into ring slot `slot` (producer waves
    // below NSIDE; one more vector-memory operation for them per tile)
    auto load_side = [&](int64_t t0, int slot) __attribute__((always_inline)) {
        if constexpr (NSIDE > 0) {
            if (wave < NSIDE) {
                const float* src = (L2 && wave == 0) ? args.yn : args.yinv;
                int64_t row = t0 + lane;
                row = row < c1 ? row : c1 - 1;
                if constexpr (VEC) {
                    dma4(src + row, (uint32_t)(uintptr_t)(lds_ptr_t)&side[wave][slot][0]);
                } else {
                    side[wave][slot][lane] = src[row];
                }
            }
        }
    };
    auto load_tile = [&](int64_t t0, int buf) __attribute__((always_inline)) {
        const uint32_t base = tile_lds(buf) + (uint32_t)(wave * 64 * 16);
        if (t0 + BN <= c1) {  // wave-uniform: a whole tile of the chunk
#pragma unroll
            for (int t = 0; t < LPW; ++t) {
                if constexpr (VEC) {
                    dma16(xb + t0 * row_bytes + loff[t], base + (uint32_t)(t * kProducers * 64 * 16));
                } else {
                    int j, cc;
                    granule_of(t, j, cc);
                    tile_buf(buf)[(wave + t * kProducers) * 64 + lane] =
                        load_granule<Op, false>(xb + (t0 + j) * row_bytes, cc, args.valid, true);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < LPW; ++t) {
                int j, cc;
                granule_of(t, j, cc);
                int64_t row = t0 + j;
                row = row < c1 ? row : c1 - 1;
                if constexpr (VEC) {
                    dma16(xb + row * row_bytes + cc * 16, base + (uint32_t)(t * kProducers * 64 * 16));
                } else {
                    tile_buf(buf)[(wave + t * kProducers) * 64 + lane] =
                        load_granule<Op, false>(xb + row * row_bytes, cc, args.valid, true);
                }
            }
        }
    };

    if (wave < kProducers) {
        // ------------------------------------------------ producer
        const int li = lane & 15, lh = lane >> 4;
        const int qg = wave / DG, dg = wave % DG;
        const unsigned char* xq = static_cast<const unsigned char*>(args.xq);
        uint4 areg[QPB][S4];
#pragma unroll
        for (int qb = 0; qb < QPB; ++qb) {
            const int64_t q = q0 + (qg * QPB + qb) * 16 + li;
            const bool ok = q < args.nq;
            const unsigned char* row = xq + (ok ? q : 0) * row_bytes;
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4) areg[qb][s4] = load_granule<Op, VEC>(row, 4 * s4 + lh, args.valid, ok);
        }
        // the A operands have landed before any tile load is issued, so no
        // wait in the step loop has to cover them
        __builtin_amdgcn_s_waitcnt(0);
        // Step barrier of the kernel: LDS writes (scores) complete, no LDS
        // access crosses it, and -- unlike a fence -- the tile loads in flight
        // are not waited for.
        auto step_barrier = [&]() __attribute__((always_inline)) {
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        };
        // all but the newest AHEAD - 1 tiles' loads done (each producer
        // wave: LPW loads per tile, one more when it loads a side array)
        auto wait_ahead = [&]() __attribute__((always_inline)) {
            if (NSIDE > 0 && wave < NSIDE)
                __builtin_amdgcn_s_waitcnt(waitcnt_vm<(AHEAD - 1) * (LPW + 1)>());
            else
                __builtin_amdgcn_s_waitcnt(waitcnt_vm<(AHEAD - 1) * LPW>());
        };
        // The first AHEAD tiles, then wait for tile 0 only.
#pragma unroll
        for (int t = 0; t < AHEAD; ++t)
            if (t < nsteps) {
                load_tile(c0 + (int64_t)t * BN, t);
                load_side(c0 + (int64_t)t * BN, t);
            }
        if (nsteps >= AHEAD)
            wait_ahead();
        else
            __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // Step s reads buffer s % NBUF and loads tile s + AHEAD into buffer
        // (s + AHEAD) % NBUF, which step s - 1 read before the last barrier.
        // The loop is unrolled NBUF times so that every buffer is named
        // statically.
        auto produce = [&](int s, int u) __attribute__((always_inline)) {
            const uint4* bt = tile_buf(u);
            // All B granules of the step first, so that LDS latency
            // overlaps the matrix work of earlier granules.
            uint4 b[S4][DPB];
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4)
#pragma unroll
                for (int db = 0; db < DPB; ++db) {
                    const int j = (dg * DPB + db) * 16 + li;
                    b[s4][db] = bt[j * GR + ((4 * s4 + lh) ^ (j & SW))];
                }
            // SK independent accumulators per output block (split over the
            // granule steps) keep at least four MFMA chains in flight.
            floatx4 acc[SK][QPB][DPB];
#pragma unroll
            for (int kk = 0; kk < SK; ++kk)
#pragma unroll
                for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                    for (int db = 0; db < DPB; ++db) acc[kk][qb][db] = floatx4{0.f, 0.f, 0.f, 0.f};
            // The tile loads AHEAD steps ahead are issued between the two
            // halves of the matrix work, so their issue cost hides under it.
            constexpr int H = S4 / 2;
#pragma unroll
            for (int s4 = 0; s4 < H; ++s4)
#pragma unroll
                for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                    for (int db = 0; db < DPB; ++db)
                        acc[s4 % SK][qb][db] = Op::mma(acc[s4 % SK][qb][db], areg[qb][s4], b[s4][db]);
            __builtin_amdgcn_sched_barrier(0);
            const bool issue = s + AHEAD < nsteps;
            if (issue) {
                load_tile(c0 + (int64_t)(s + AHEAD) * BN, (u + AHEAD) % NBUF);
                load_side(c0 + (int64_t)(s + AHEAD) * BN, (s + AHEAD) % (NBUF + 1));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s4 = H; s4 < S4; ++s4)
#pragma unroll
                for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                    for (int db = 0; db < DPB; ++db)
                        acc[s4 % SK][qb][db] = Op::mma(acc[s4 % SK][qb][db], areg[qb][s4], b[s4][db]);
            // D[i][j] of a 16x16 block sits in lane j + 16*(i/4), element
            // i%4: one 16-byte store of queries 4*lh .. 4*lh+3 of column j.
            float* slot = scores[s & 1];
#pragma unroll
            for (int qb = 0; qb < QPB; ++qb)
#pragma unroll
                for (int db = 0; db < DPB; ++db) {
                    floatx4 v = acc[0][qb][db];
#pragma unroll
                    for (int kk = 1; kk < SK; ++kk) v += acc[kk][qb][db];
                    const int j = (dg * DPB + db) * 16 + li;
                    *reinterpret_cast<floatx4*>(&slot[j * LDQ + (qg * QPB + qb) * 16 + 4 * lh]) = v;
                }
            // the next step's tile must have landed (this wave's part of it;
            // the barrier covers the other producers); the AHEAD - 1 tiles
            // after it stay in flight
            if (issue)
                wait_ahead();
            else
                __builtin_amdgcn_s_waitcnt(0);
        };
#pragma unroll 1
        for (int s0 = 0; s0 <= nsteps; s0 += NBUF) {
#pragma unroll
            for (int u = 0; u < NBUF; ++u) {
                const int s = s0 + u;
                if (s <= nsteps) {
                    if (s < nsteps) produce(s, u);
                    step_barrier();
                }
            }
        }
    } else {
        // ------------------------------------------------ consumer
        // score = ||y||^2 - 2 q.y (L2) or -q.y (inner product); ||x||^2 is the
        // same for every candidate of a query and does not change its rank.
        // Scaled formats multiply q.y by the query's and the row's 1/scale.
        // The pool selectors take the consumer index from the thread id
        // (vector registers): made scalar, their wave-uniform state outgrows
        // the scalar registers and spills.
        const int cw = S::mem_queues ? (int)(threadIdx.x >> 6) - kProducers : wave - kProducers;
        using Sel = typename std::conditional<S::mem_queues, PoolSelect<KR, QW, NBINS>,
                                              MultiSelect<KR, T, QW>>::type;
        Sel sel;
        const int64_t qf = q0 + cw * QW;
        const int64_t left = args.nq - qf;
        const int nvalid = (int)(left < 0 ? 0 : left < QW ? left : QW);
        uint32_t* ranks =
            args.bound && left > 0 ? args.bound + (qf * args.nchunks + chunk) * kRankPoints : nullptr;
        if constexpr (S::mem_queues) {
            sel.init(args.keff, args.part + (qf * args.nchunks + chunk) * S::ROW,
                     (int64_t)args.nchunks * S::ROW, nvalid, ranks, args.nchunks,
                     bins[S::mem_queues ? cw : 0], args.drops);
        } else {
            sel.init(args.keff, nvalid, ranks, args.nchunks);
        }
        float qs[QW];
#pragma unroll
        for (int qq = 0; qq < QW; ++qq) {
            const int64_t q = q0 + cw * QW + qq;
            qs[qq] = (Op::SCALED && q < args.nq) ? args.qinv[q] : 1.f;
        }
        __syncthreads();
        // bound exchanges: often early, while the queues fill (steps 0, 4, 8,
        // 16, 32), then every 64 steps
        int next_x = args.bound ? 0 : nsteps + 1;
        for (int s = 0; s <= nsteps; ++s) {
            if (s == next_x) {
                next_x = s == 0 ? 4 : s < 64 ? 2 * s : s + 64;
                if constexpr (S::mem_queues)
                    exchange_ranks_wide(sel, args.bound, args.nchunks, qf, args.nq);
                else
                    exchange_ranks(sel, args.bound, args.nchunks, qf, args.nq);
            }
            if (s >= 1) {
                if constexpr (S::mem_queues) {
                    // consumers' urgency flags of the previous step
                    bool batch = false;
                    if constexpr (Sel::kBatch) {
                        if (s >= 2) {
#pragma unroll
                            for (int c = 0; c < S::NC; ++c) batch |= urgent_flags[s & 1][c] != 0u;
                        }
                    }
                    sel.refine_pools(batch);
                }
                const float* slot = scores[(s - 1) & 1];
                const int64_t g = c0 + (int64_t)(s - 1) * BN + lane;
                const bool ok = g < c1;
                // side values of step s - 1's tile (landed before the barrier
                // that ended step s - 2; overwritten only after this step)
                const int ring = (s - 1) % (NBUF + 1);
                const float ynv = L2 ? side[0][ring][lane] : 0.f;
                const float ysv = Op::SCALED ? side[L2 ? 1 : 0][ring][lane] : 1.f;
                float score[QW];
                const float* col = slot + lane * LDQ + cw * QW;
                if constexpr (QW % 4 == 0) {
#pragma unroll
                    for (int qq = 0; qq < QW; qq += 4) {
                        const floatx4 cc = *reinterpret_cast<const floatx4*>(col + qq);
#pragma unroll
                        for (int e = 0; e < 4; ++e) score[qq + e] = cc[e];
                    }
                } else {
#pragma unroll
                    for (int qq = 0; qq < QW; qq += 2) {
                        const float2 cc = *reinterpret_cast<const float2*>(col + qq);
                        score[qq] = cc.x;
                        score[qq + 1] = cc.y;
                    }
                }
#pragma unroll
                for (int qq = 0; qq < QW; ++qq) {
                    float c = score[qq];
                    if (Op::SCALED) c = c * qs[qq] * ysv;
                    score[qq] = L2 ? fmaf(-2.f, c, ynv) : -c;
                }
                sel.offer(score, (uint32_t)g, ok);
                if constexpr (S::mem_queues) {
                    if constexpr (Sel::kBatch) {
                        const bool u = sel.urgent();
                        if (lane == 0) urgent_flags[(s + 1) & 1][cw] = u ? 1u : 0u;
                    }
                }
            }
            // the producers' step barrier (LDS only: the consumers' own
            // global loads and pool appends are not waited for here)
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        }
        sel.finish();
        if constexpr (!S::mem_queues) {
#pragma unroll
            for (int qq = 0; qq < QW; ++qq) {
                const int64_t q = q0 + cw * QW + qq;
                if (q < args.nq) {
                    uint64_t* out = args.part + (q * args.nchunks + chunk) * S::ROW;
#pragma unroll
                    for (int r = 0; r < KR; ++r) out[r * 64 + lane] = sel.key(qq, r);
                }
            }
        }
    }
}

static __global__ void fill_bounds_kernel(uint32_t* __restrict__ bound, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bound[i] = v;
}

// Words of the rank-point array of a search with nchunks chunks.
inline int64_t bound_words(int KR, int64_t nq, int64_t nchunks) {
    (void)KR;
    return nq * nchunks * kRankPoints;
}

// No rank point yet: "no rows proven" (kNoBound).
inline mk_status clear_bounds(int KR, uint32_t* bound, int64_t nq, int64_t nchunks, hipStream_t s) {
    const int64_t n = bound_words(KR, nq, nchunks);
    if (n == 0) return MK_OK;
    hipLaunchKernelGGL(fill_bounds_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, bound,
                       n, kNoBound);
    MK_LAUNCHED();
    return MK_OK;
}

// Chunking of the database.  Chunks of a query that run at the same time
// each fill their queue before shared bounds can help, and a pool's
// insertions grow with the number of chunks, so long queues get few, long
// chunks: about 2 workgroups per CU for queues of 512+ entries, 16
// otherwise, chunks of at least 32 queue lengths (8 for short queues when
// that would leave most CUs idle), at most kMaxRankChunks chunks, and among
// chunk counts within 25% of that target the one whose last wave of
// workgroups is fullest.
inline void plan_chunks(int64_t nq, int64_t nb, int BQ, int BN, int KS, int64_t* nqb,
                        int64_t* nchunks, int64_t* chunk_len) {
    constexpr int64_t kCUs = 256;
    *nqb = ceil_div(nq, BQ);
    const int64_t target = (KS >= 512 ? 2 : 16) * kCUs;
    const int64_t want = ceil_div(target, *nqb);
    // short queues (128 entries or fewer) over a database that gives fewer
    // than kCUs / 2 workgroups at 32 queue lengths per chunk (a small batch
    // against IVF coarse centroids): chunks of 8 queue lengths, since then
    // the sweep's step count, not the insertions, sets the time
    const int64_t min_len =
        (KS <= 128 && *nqb * (nb / (32 * KS)) < kCUs / 2) ? 8 * (int64_t)KS : 32 * (int64_t)KS;
    int64_t max_by_len = nb / min_len > 1 ? nb / min_len : 1;
    if (max_by_len > kMaxRankChunks) max_by_len = kMaxRankChunks;
    int64_t hi = want < max_by_len ? want : max_by_len;
    if (hi < 1) hi = 1;
    int64_t lo = (hi * 3) / 4 > 1 ? (hi * 3) / 4 : 1;
    int64_t nc = hi;
    double best = -1.0;
    for (int64_t c = hi; c >= lo; --c) {
        const int64_t wgs = *nqb * c;
        const double fill = (double)wgs / (double)(ceil_div(wgs, kCUs) * kCUs);
        if (fill > best + 1e-9) {
            best = fill;
            nc = c;
        }
    }
    int64_t cl = ceil_div(ceil_div(nb, nc), BN) * BN;
    if (cl == 0) cl = BN;
    *chunk_len = cl;
    *nchunks = nb > 0 ? ceil_div(nb, cl) : 1;
}

constexpr int kMergeWaves = 4;
constexpr int kMaxDim = 512;

// FP32 direct-form squared distances (l2) or inner products of the query row
// xw (in LDS) to the database rows named by one wave's keys kl[e], e in
// [e0, e0 + 16), written to dist[e] for e < keff (sentinel keys: 0).  16
// lanes per row and 4 rows per pass, each lane summing every 16th 16-byte
// granule of the row (coalesced), then a 16-lane reduction; the four passes'
// row loads are in flight together (the gathers are latency-bound one pass
// at a time).
__device__ __forceinline__ void rerank_rows16(const float* xw, const uint64_t* kl, int e0,
                                              int keff, const float* __restrict__ xb, int32_t d,
                                              int32_t vec, int32_t l2, float* dist) {
    constexpr int NP = 4;
    const int lane = lane_id();
    const int sub = lane & 15, rsel = lane >> 4;
    const float* y[NP];
    bool live[NP];
    float sacc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int e = e0 + 4 * p + rsel;
        const uint64_t key = e < keff ? kl[e] : kSentinel;
        live[p] = key != kSentinel;
        y[p] = xb + (int64_t)(live[p] ? key_index(key) : 0u) * d;
        sacc[p] = 0.f;
    }
    if (vec) {
        for (int t = 4 * sub; t < d; t += 64) {
            float4 yv[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p)
                yv[p] = live[p] ? *reinterpret_cast<const float4*>(y[p] + t) : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 xv = *reinterpret_cast<const float4*>(xw + t);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (l2) {
                    const float a = xv.x - yv[p].x, b = xv.y - yv[p].y, c = xv.z - yv[p].z,
                                dd = xv.w - yv[p].w;
                    sacc[p] = fmaf(a, a, sacc[p]);
                    sacc[p] = fmaf(b, b, sacc[p]);
                    sacc[p] = fmaf(c, c, sacc[p]);
                    sacc[p] = fmaf(dd, dd, sacc[p]);
                } else {
                    sacc[p] = fmaf(xv.x, yv[p].x, sacc[p]);
                    sacc[p] = fmaf(xv.y, yv[p].y, sacc[p]);
                    sacc[p] = fmaf(xv.z, yv[p].z, sacc[p]);
                    sacc[p] = fmaf(xv.w, yv[p].w, sacc[p]);
                }
            }
        }
    } else {
        for (int t = sub; t < d; t += 16) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float yt = live[p] ? y[p][t] : 0.f;
                if (l2) {
                    const float a = xw[t] - yt;
                    sacc[p] = fmaf(a, a, sacc[p]);
                } else {
                    sacc[p] = fmaf(xw[t], yt, sacc[p]);
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float v = live[p] ? sacc[p] : 0.f;
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
        const int e = e0 + 4 * p + rsel;
        if (sub == 0 && e < keff) dist[e] = v;
    }
}


// The first k of a wave's sorted (score, row) keys as distances (L2) or
// inner products and row ids; sentinels become (+-inf, -1).
template <int KR>
__device__ __forceinline__ void emit_reranked(const uint64_t (&nk)[KR], int32_t k, int32_t l2,
                                              float* __restrict__ Dq, int64_t* __restrict__ Iq) {
    const int lane = lane_id();
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        if (e < k) {
            const uint64_t key = nk[r];
            if (key == kSentinel) {
                Dq[e] = l2 ? INFINITY : -INFINITY;
                Iq[e] = -1;
            } else {
                const float s = key_score(key);
                Dq[e] = l2 ? s : -s;
                Iq[e] = (int64_t)key_index(key);
            }
        }
    }
}

template <int KR>
__global__ __launch_bounds__(64 * kMergeWaves) void knn_merge_rerank(
    const uint64_t* __restrict__ part, int32_t nchunks, int32_t row, int32_t nread,
    const float* __restrict__ xq, int64_t nq,
    const float* __restrict__ xb, int32_t d, int32_t vec, int32_t l2, int32_t k, int32_t keff,
    float* __restrict__ D, int64_t* __restrict__ I) {
    constexpr int T = SelParams<KR>::T;
    constexpr int KS = 64 * KR;
    __shared__ __align__(16) float xs[kMergeWaves][kMaxDim];
    __shared__ uint64_t kl[kMergeWaves][KS];
    __shared__ float dist[kMergeWaves][KS];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kMergeWaves + wave;
    if (q >= nq) return;

    WaveSelect<KR, T> ws;
    ws.init(keff);
    const uint64_t* p = part + q * nchunks * row;
    // The first nread entries of each chunk's row hold its candidates (a
    // sorted list needs only its first keff).
    const int per = (nread + 63) & ~63;
#pragma unroll 1
    for (int c = 0; c < nchunks; ++c) {
#pragma unroll 1
        for (int e = 0; e < per; e += 64) {
            const int i = e + lane;
            if (ws.push(i < nread ? p[(int64_t)c * row + i] : kSentinel)) ws.merge();
        }
    }
    ws.finish();

    const float* x = xq + q * d;
    for (int t = lane; t < d; t += 64) xs[wave][t] = x[t];
    // the kept keys, in list order, through LDS
#pragma unroll
    for (int r = 0; r < KR; ++r) kl[wave][r * 64 + lane] = ws.w[r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");

    // exact distances of the first keff keys, 16 rows per step
    const float* xw = xs[wave];
#pragma unroll 1
    for (int e0 = 0; e0 < keff; e0 += 16)
        rerank_rows16(xw, kl[wave], e0, keff, xb, d, vec, l2, dist[wave]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");

    uint64_t nk[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const uint64_t key = ws.w[r];
        const int e = r * 64 + lane;
        nk[r] = kSentinel;
        if (key != kSentinel && e < keff) {
            const float sv = dist[wave][e];
            nk[r] = make_key(l2 ? sv : -sv, key_index(key));
        }
    }
    bitonic_sort<false, KR>(nk);
    emit_reranked<KR>(nk, k, l2, D + q * k, I + q * k);
}

// Exact re-rank of one query's short list (the first R keys of its row of
// 64 * KR) by a whole workgroup: the waves share the rows' exact distances,
// 16 rows per wave per step, then wave 0 sorts the (distance, row) keys and
// writes the first k.  The same rows, distances and final sort as
// knn_merge_rerank over one chunk of R, so the same results, with a quarter
// of its gather latency per query.
template <int KR>
__global__ __launch_bounds__(64 * kMergeWaves) void knn_rerank_block(
    const uint64_t* __restrict__ keys, int32_t R, const float* __restrict__ xq,
    const float* __restrict__ xb, int32_t d, int32_t vec, int32_t l2, int32_t k,
    float* __restrict__ D, int64_t* __restrict__ I) {
    constexpr int KS = 64 * KR;
    __shared__ __align__(16) float xs[kMaxDim];
    __shared__ uint64_t kl[KS];
    __shared__ float dist[KS];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t q = blockIdx.x;
    const uint64_t* p = keys + q * KS;
    for (int e = threadIdx.x; e < KS; e += 64 * kMergeWaves) kl[e] = e < R ? p[e] : kSentinel;
    for (int t = threadIdx.x; t < d; t += 64 * kMergeWaves) xs[t] = xq[q * d + t];
    __syncthreads();
#pragma unroll 1
    for (int e0 = 16 * wave; e0 < R; e0 += 16 * kMergeWaves)
        rerank_rows16(xs, kl, e0, R, xb, d, vec, l2, dist);
    __syncthreads();
    if (wave != 0) return;
    uint64_t nk[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        const uint64_t key = kl[e];
        nk[r] = kSentinel;
        if (key != kSentinel && e < R) {
            const float sv = dist[e];
            nk[r] = make_key(l2 ? sv : -sv, key_index(key));
        }
    }
    bitonic_sort<false, KR>(nk);
    emit_reranked<KR>(nk, k, l2, D + q * k, I + q * k);
}


}  // namespace mk
