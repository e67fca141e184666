// Register-resident k-selection for 64-lane wavefronts (gfx950).
//
// This is the selection design of Section 4 (WarpSelect, Algorithm 3) rebuilt
// for CDNA's wave64:
//   * keys are 64-bit: an order-preserving transform of the FP32 distance in
//     the high word, the candidate index in the low word, so a single
//     unsigned compare orders by (distance, index) -- the lower index wins
//     ties, which the paper leaves unspecified;
//   * the wave queue W is a lane-stride register array (Section 3.2): element
//     i sits in lane i % 64 of register i / 64, KR registers, ascending;
//   * each lane has a thread queue of T slots, filled in arrival order with
//     candidates that beat the current k-th best key (a tighter filter than
//     the thread-queue head of Algorithm 3: only candidates that can enter
//     the result are kept);
//   * when any lane's thread queue is full (a wave ballot), the 64*T thread
//     queue entries are sorted by a bitonic network (Section 4.1) into
//     descending order, merged into W by the inverted first stage of the
//     odd-size merge of Algorithm 1 (pairing W[i] with the thread array
//     counted from its end, which lands in the same lane and needs no
//     shuffle), and W is re-sorted by a bitonic half-cleaner cascade; the
//     thread queues are then emptied (everything not kept is provably outside
//     the k best seen so far).
// Cross-lane compare-exchange uses DPP quad permutes for strides 1 and 2,
// ds_swizzle for strides 4..16 and ds_bpermute for stride 32; strides that
// are multiples of 64 stay inside a lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

constexpr uint64_t kSentinel = ~0ull;

// Order-preserving map of FP32 bits to uint32 (negative values flip all bits,
// non-negative values set the sign bit).  -0.0 must be canonicalised before.
__device__ __forceinline__ uint32_t float_order(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t mask = (uint32_t)((int32_t)u >> 31) | 0x80000000u;
    return u ^ mask;
}

__device__ __forceinline__ float order_float(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
    return __uint_as_float(u);
}

// Key of a candidate whose smaller score is better.
__device__ __forceinline__ uint64_t make_key(float score, uint32_t idx) {
    score = score + 0.0f;  // -0.0 -> +0.0 so that zero ties go by index
    return ((uint64_t)float_order(score) << 32) | idx;
}

__device__ __forceinline__ float key_score(uint64_t key) { return order_float((uint32_t)(key >> 32)); }
__device__ __forceinline__ uint32_t key_index(uint64_t key) { return (uint32_t)key; }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Value held by lane (lane ^ S).
template <int S>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v) {
    static_assert(S >= 1 && S <= 32 && (S & (S - 1)) == 0, "stride must be a power of two");
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (S < 32) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (S << 10));
    } else {
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, (int)v);
    }
}

template <int S>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
    uint32_t lo = xor_lane32<S>((uint32_t)v);
    uint32_t hi = xor_lane32<S>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// One compare-exchange layer of a bitonic network over a lane-stride array of
// R registers: element i is paired with i ^ S; the pair is put in ascending
// order when bit P of i is clear (descending when set), all flipped if DESC.
template <int P, int S, bool DESC, int R>
__device__ __forceinline__ void cx_layer(uint64_t (&v)[R]) {
    if constexpr (S >= 64) {
        constexpr int RS = S / 64;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if ((r & RS) == 0) {
                const int r2 = r | RS;
                const bool up = (((r * 64) & P) == 0) != DESC;
                uint64_t a = v[r], b = v[r2];
                uint64_t lo = umin64(a, b), hi = umax64(a, b);
                v[r] = up ? lo : hi;
                v[r2] = up ? hi : lo;
            }
        }
    } else {
        const int lane = lane_id();
        const bool lower = (lane & S) == 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bool up;
            if constexpr (P >= 64) {
                up = (((r * 64) & P) == 0) != DESC;
            } else {
                up = ((lane & P) == 0) != DESC;
            }
            uint64_t p = xor_lane64<S>(v[r]);
            const bool keep_min = (lower == up);
            v[r] = keep_min ? umin64(v[r], p) : umax64(v[r], p);
        }
    }
}

// Half-cleaner cascade with strides S, S/2, ..., 1 at block size P.
template <int P, int S, bool DESC, int R>
__device__ __forceinline__ void cx_cascade(uint64_t (&v)[R]) {
    if constexpr (S >= 1) {
        cx_layer<P, S, DESC, R>(v);
        cx_cascade<P, S / 2, DESC, R>(v);
    }
}

template <int P, int N, bool DESC, int R>
__device__ __forceinline__ void bitonic_sort_from(uint64_t (&v)[R]) {
    if constexpr (P <= N) {
        cx_cascade<P, P / 2, DESC, R>(v);
        bitonic_sort_from<P * 2, N, DESC, R>(v);
    }
}

// Full bitonic sort of the 64*R-element lane-stride array (R a power of two).
template <bool DESC, int R>
__device__ __forceinline__ void bitonic_sort(uint64_t (&v)[R]) {
    static_assert((R & (R - 1)) == 0, "register count must be a power of two");
    bitonic_sort_from<2, 64 * R, DESC, R>(v);
}

// Sort a bitonic 64*R-element array ascending.
template <int R>
__device__ __forceinline__ void bitonic_clean(uint64_t (&v)[R]) {
    cx_cascade<64 * R, 32 * R, false, R>(v);
}

// Merge the (unsorted) thread-queue array tq into the ascending wave queue w,
// keeping the 64*KR smallest keys of both, then empty tq.
template <int KR, int T>
__device__ __forceinline__ void ws_merge(uint64_t (&w)[KR], uint64_t (&tq)[T]) {
    bitonic_sort<true, T>(tq);  // descending
    if constexpr (KR >= T) {
#pragma unroll
        for (int r = KR - T; r < KR; ++r) w[r] = umin64(w[r], tq[r - (KR - T)]);
    } else {
#pragma unroll
        for (int r = 0; r < KR; ++r) w[r] = umin64(w[r], tq[r + (T - KR)]);
    }
    bitonic_clean<KR>(w);
#pragma unroll
    for (int i = 0; i < T; ++i) tq[i] = kSentinel;
}

// Hide a register value from the optimiser.  A chain of selects between
// array elements keyed on a runtime index is otherwise folded back into an
// indexed load, which forces the whole register array into scratch memory.
__device__ __forceinline__ uint64_t opaque(uint64_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Element `pos` (wave-uniform, < 64*KR) of a lane-stride array.
template <int KR>
__device__ __forceinline__ uint64_t ws_element(const uint64_t (&w)[KR], int pos) {
    const int reg = pos >> 6;
    const int lane = pos & 63;
    uint64_t v = opaque(w[0]);
#pragma unroll
    for (int r = 1; r < KR; ++r) {
        const uint64_t e = opaque(w[r]);
        v = r == reg ? e : v;
    }
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// The thread queues of a wave form one buffer of 64*T keys in lane-stride
// order (position p in register p / 64 of lane p % 64) that is filled densely:
// the keys of the lanes whose `take` is set (`bal` = their ballot) go to
// positions count, count + 1, ... in lane order, moved there by one forward
// permute (lanes without a key are sent to the remaining lanes, so the
// permute is a bijection).  Order inside the buffer does not matter, the merge
// sorts it.  Returns the new count; count + popcount(bal) <= 64*T.
template <int T>
__device__ __forceinline__ int tq_append(uint64_t (&tq)[T], uint64_t key, bool take,
                                         uint64_t bal, int count) {
    const int lane = lane_id();
    const int n = __popcll(bal);
    const int below = (int)__builtin_amdgcn_mbcnt_hi(
        (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    const int base = count & 63;
    const int dst = take ? (base + below) & 63 : (base + n + (lane - below)) & 63;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)key);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)(key >> 32));
    const uint64_t got = ((uint64_t)hi << 32) | lo;
    const int rel = (lane - base) & 63;  // this lane holds position count + rel
    const bool valid = rel < n;
    const int reg = (count + rel) >> 6;
#pragma unroll
    for (int i = 0; i < T; ++i) tq[i] = (valid && reg == i) ? got : tq[i];
    return count + n;
}

// Single-stream selector: one wave selects the `keff` smallest keys of a
// stream offered 64 keys (one per lane) at a time.  Must be used by all
// lanes of the wave in uniform control flow.  push() only fills thread
// queues and reports whether a merge is due; callers keep a single merge()
// call site so that the merge network is emitted once per kernel.
template <int KR, int T>
struct WaveSelect {
    uint64_t w[KR];
    uint64_t tq[T];
    uint64_t kth;   // current keff-th smallest key (sentinel until W holds keff)
    float kth_f;    // its score; +inf while kth is the sentinel
    int keff;
    int cnt;        // keys in the thread-queue buffer (wave-uniform)

    __device__ __forceinline__ void init(int k_eff) {
#pragma unroll
        for (int r = 0; r < KR; ++r) w[r] = kSentinel;
#pragma unroll
        for (int i = 0; i < T; ++i) tq[i] = kSentinel;
        kth = kSentinel;
        kth_f = INFINITY;
        keff = k_eff;
        cnt = 0;
    }

    __device__ __forceinline__ void merge() {
        ws_merge<KR, T>(w, tq);
        cnt = 0;
        kth = ws_element<KR>(w, keff - 1);
        kth_f = kth == kSentinel ? INFINITY : key_score(kth);
    }

    // Offer one key per lane; returns true (wave-uniform) when a merge is due
    // (the buffer might not hold another 64 keys).
    __device__ __forceinline__ bool push(uint64_t key) {
        const bool take = key < kth;
        const uint64_t bal = __ballot(take);
        if (bal) {
            cnt = tq_append<T>(tq, key, take, bal, cnt);
            return cnt > 64 * (T - 1);
        }
        return false;
    }

    // A score that cannot beat the current keff-th key (strictly worse than
    // its score) can be discarded without building its key.
    __device__ __forceinline__ bool may_take(float score) const { return score <= kth_f; }

    __device__ __forceinline__ void finish() { merge(); }
};

}  // namespace mk
