// Row-wise k-selection of a resident matrix (Section 2 problem statement,
// Section 4.2 selection, Section 6.1 benchmark shape) and the generic merge of
// per-segment partial results (the second pass of the two-pass k-selection of
// Section 5.3).
//
// Pass 1: one wave per (row, segment) streams the segment once with 16-byte
// coalesced loads and feeds WaveSelect.  A row that fits one segment writes
// its final result directly; otherwise the wave writes its k best keys and
// pass 2 (one wave per row) selects over the segments' keys.
#include "common.hpp"
#include "fused.hpp"
#include "kselect.hpp"
#include "profile.hpp"
#include "wave_select.hpp"

namespace mk {

namespace {

constexpr int kWavesPerBlock = 4;

template <bool LARGEST>
__device__ __forceinline__ uint64_t value_key(float v, uint32_t idx) {
    return make_key(LARGEST ? -v : v, idx);
}

// Write the first k keys of a lane-stride queue as (value, index) pairs.
template <int KR, bool LARGEST>
__device__ __forceinline__ void emit_values(const uint64_t (&w)[KR], int k, float* vals,
                                            int64_t* idx) {
    const int lane = lane_id();
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        if (e < k) {
            const uint64_t key = w[r];
            if (key == kSentinel) {
                vals[e] = LARGEST ? -INFINITY : INFINITY;
                idx[e] = -1;
            } else {
                const float s = key_score(key);
                vals[e] = LARGEST ? -s : s;
                idx[e] = (int64_t)key_index(key);
            }
        }
    }
}

template <int KR>
__device__ __forceinline__ void emit_keys(const uint64_t (&w)[KR], int k, uint64_t* out) {
    const int lane = lane_id();
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int e = r * 64 + lane;
        if (e < k) out[e] = w[r];
    }
}

template <int KR, int T, bool LARGEST>
__global__ __launch_bounds__(64 * kWavesPerBlock) void kselect_pass1(
    const float* __restrict__ a, int64_t nrows, int64_t len, int32_t k, int32_t nseg,
    int64_t seg_len, float* __restrict__ vals, int64_t* __restrict__ idx,
    uint64_t* __restrict__ partial) {
    constexpr int U = 4;  // float4 loads in flight per lane
    __shared__ float stage[kWavesPerBlock][4 * U][64];
    const int wave = threadIdx.x / 64;
    const int lane = lane_id();
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (unit >= nrows * (int64_t)nseg) return;  // wave-uniform
    const int64_t row = unit / nseg;
    const int64_t seg = unit % nseg;
    const int64_t lo = seg * seg_len;
    const int64_t hi = lo + seg_len < len ? lo + seg_len : len;
    const float* rp = a + row * len;

    WaveSelect<KR, T> ws;
    ws.init(k);

    // Vector body over 16-byte aligned rows: lane takes 4 consecutive values
    // per load, U loads in flight.  Most groups are rejected by one compare
    // per value against the current k-th score; a group with any candidate
    // is staged in LDS and offered value by value from a single loop, so the
    // merge network appears once in the kernel.
    const bool aligned = (reinterpret_cast<uintptr_t>(rp + lo) & 15) == 0;
    const int64_t vec_end = aligned ? lo + ((hi - lo) / (256 * U)) * (256 * U) : lo;
    for (int64_t e = lo; e < vec_end; e += 256 * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = *reinterpret_cast<const float4*>(rp + e + u * 256 + lane * 4);
        bool cand = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cand |= ws.may_take(LARGEST ? -v[u].x : v[u].x);
            cand |= ws.may_take(LARGEST ? -v[u].y : v[u].y);
            cand |= ws.may_take(LARGEST ? -v[u].z : v[u].z);
            cand |= ws.may_take(LARGEST ? -v[u].w : v[u].w);
        }
        if (__any(cand)) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                stage[wave][4 * u + 0][lane] = v[u].x;
                stage[wave][4 * u + 1][lane] = v[u].y;
                stage[wave][4 * u + 2][lane] = v[u].z;
                stage[wave][4 * u + 3][lane] = v[u].w;
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int j = 0; j < 4 * U; ++j) {
                const float val = stage[wave][j][lane];
                const uint32_t i = (uint32_t)(e + (j >> 2) * 256 + lane * 4 + (j & 3));
                if (ws.push(value_key<LARGEST>(val, i))) ws.merge();
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    // Scalar remainder (and unaligned rows): one value per lane per step.
#pragma unroll 1
    for (int64_t e = vec_end; e < hi; e += 64) {
        const int64_t i = e + lane;
        const uint64_t key = i < hi ? value_key<LARGEST>(rp[i], (uint32_t)i) : kSentinel;
        if (ws.push(key)) ws.merge();
    }
    ws.finish();
    if (nseg == 1) {
        emit_values<KR, LARGEST>(ws.w, k, vals + row * k, idx + row * k);
    } else {
        emit_keys<KR>(ws.w, k, partial + unit * k);
    }
}

// Pass 1 for queues of 256+ entries: a sorted queue is the wrong structure
// there (every merge runs a network over the whole queue for a buffer of
// new keys), so candidates that beat the current threshold are appended to
// an unsorted pool of 2 * 64 * KR keys in device memory, cut back by a
// radix selection inside the wave whenever it nears capacity (PoolSelect,
// the fused search's selector).  At the end the pool is cut to 64 * KR keys,
// which one WaveSelect pass sorts.
//
// Most of a segment would be offered early, while the pool's threshold is
// still loose, so the threshold starts from a guess: the score of rank
// about 1.5 k SN / L + 32 among the segment's first SN = 8192 scores (a
// 512-bin histogram over their range), which about 1.5 k of the L scores
// beat when the prefix is typical.  Values at or below the guess (and the
// pool's own threshold) are appended in bulk: a lane counts its candidates
// among its 16 values, a wave prefix sum places them, and each lane writes
// its own.  The guess is no bound, so it is checked: when fewer than k
// values were appended, fewer than k scores lie at or below it and the
// segment is streamed again without it (the plain pool selection).
// Otherwise the k best scores are all at or below it and the result is
// exact.
template <int KR, bool LARGEST>
__global__ __launch_bounds__(64 * kWavesPerBlock) void kselect_pool(
    const float* __restrict__ a, int64_t nrows, int64_t len, int32_t k, int32_t nseg,
    int64_t seg_len, float* __restrict__ vals, int64_t* __restrict__ idx,
    uint64_t* __restrict__ partial, uint64_t* __restrict__ pools,
    unsigned long long* drops) {
    constexpr int U = 4;
    constexpr int NB = 512;
    constexpr int SN = 8192;  // prefix that yields the guess
    constexpr int T = SelParams<KR>::T;
    // cuts load 8 pool rows per lane at a time: few registers, so that
    // enough waves stream the input
    using Pool = PoolSelect<KR, 1, NB, 8>;
    __shared__ float stage[kWavesPerBlock][4 * U][64];
    __shared__ uint32_t bins[kWavesPerBlock][NB];
    const int wave = threadIdx.x / 64;
    const int lane = lane_id();
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (unit >= nrows * (int64_t)nseg) return;  // wave-uniform
    const int64_t row = unit / nseg;
    const int64_t seg = unit % nseg;
    const int64_t lo = seg * seg_len;
    const int64_t hi = lo + seg_len < len ? lo + seg_len : len;
    const float* rp = a + row * len;
    uint64_t* pool_keys = pools + unit * Pool::CAP;
    auto score = [&](float v) __attribute__((always_inline)) { return LARGEST ? -v : v; };

    const bool aligned = (reinterpret_cast<uintptr_t>(rp + lo) & 15) == 0;
    const int64_t vec_end = aligned ? lo + ((hi - lo) / (256 * U)) * (256 * U) : lo;

    // ---- the guess (aligned segments of at least 4 SN values)
    float guess = INFINITY;
    if (aligned && hi - lo >= 4 * (int64_t)SN) {
        uint32_t omin = ~0u, omax = 0u;
#pragma unroll 4
        for (int t = 0; t < SN / 256; ++t) {
            const float4 v = *reinterpret_cast<const float4*>(rp + lo + t * 256 + lane * 4);
            const uint32_t o0 = float_order(score(v.x) + 0.f), o1 = float_order(score(v.y) + 0.f);
            const uint32_t o2 = float_order(score(v.z) + 0.f), o3 = float_order(score(v.w) + 0.f);
            omin = min(min(omin, min(o0, o1)), min(o2, o3));
            omax = max(max(omax, max(o0, o1)), max(o2, o3));
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            omin = min(omin, (uint32_t)__shfl_xor((int)omin, o));
            omax = max(omax, (uint32_t)__shfl_xor((int)omax, o));
        }
        const uint32_t range = omax - omin;
        const int bits = range ? 32 - __builtin_clz(range) : 0;
        const int shift = bits > 9 ? bits - 9 : 0;
        uint32_t* h = bins[wave];
#pragma unroll
        for (int j = 0; j < NB / 64; ++j) h[lane * (NB / 64) + j] = 0u;
#pragma unroll 4
        for (int t = 0; t < SN / 256; ++t) {
            const float4 v = *reinterpret_cast<const float4*>(rp + lo + t * 256 + lane * 4);
            atomicAdd(&h[(float_order(score(v.x) + 0.f) - omin) >> shift], 1u);
            atomicAdd(&h[(float_order(score(v.y) + 0.f) - omin) >> shift], 1u);
            atomicAdd(&h[(float_order(score(v.z) + 0.f) - omin) >> shift], 1u);
            atomicAdd(&h[(float_order(score(v.w) + 0.f) - omin) >> shift], 1u);
        }
        __builtin_amdgcn_s_waitcnt(waitcnt_lgkm0());
        // rank of the guess among the SN prefix scores
        const int64_t want = (3 * (int64_t)k * SN) / (2 * (hi - lo)) + 32;
        constexpr int NBL = NB / 64;
        int c[NBL], tot = 0;
#pragma unroll
        for (int j = 0; j < NBL; ++j) {
            c[j] = (int)h[lane * NBL + j];
            tot += c[j];
            h[lane * NBL + j] = 0u;  // the pool expects zeroed bins
        }
        const int incl = wave_inclusive_sum(tot);
        const uint64_t m = __ballot(incl - tot < want && want <= incl);
        if (m) {
            const int L = __builtin_ctzll(m);
            int run = incl - tot, jb = NBL - 1;
            bool f = false;
#pragma unroll
            for (int j = 0; j < NBL; ++j) {
                run += c[j];
                if (!f && run >= want) {
                    jb = j;
                    f = true;
                }
            }
            const uint32_t b = (uint32_t)(L * NBL + __builtin_amdgcn_readlane(jb, L));
            const uint64_t edge = (uint64_t)omin + (((uint64_t)b + 1) << shift) - 1;
            guess = order_float(edge >= omax ? omax : (uint32_t)edge);
        }
    }

    Pool pool;
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
        pool.init(k, pool_keys, 0, 1, nullptr, 1, bins[wave], drops);
        int appended = 0;
        auto offer = [&](float v, uint32_t i, bool ok) __attribute__((always_inline)) {
            pool.refine_pools(false);  // room for the up to 64 keys one offer appends
            const float sc[1] = {score(v)};
            const int before = pool.cnt[0];
            pool.offer(sc, i, ok && score(v) <= guess);
            appended += pool.cnt[0] - before;
        };
        for (int64_t e = lo; e < vec_end; e += 256 * U) {
            float4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = *reinterpret_cast<const float4*>(rp + e + u * 256 + lane * 4);
            const float th = fminf(guess, pool.kf[0]);
            int c = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c += score(v[u].x) <= th;
                c += score(v[u].y) <= th;
                c += score(v[u].z) <= th;
                c += score(v[u].w) <= th;
            }
            const int incl = wave_inclusive_sum(c);
            const int total = __builtin_amdgcn_readlane(incl, 63);
            if (total == 0) continue;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                stage[wave][4 * u + 0][lane] = v[u].x;
                stage[wave][4 * u + 1][lane] = v[u].y;
                stage[wave][4 * u + 2][lane] = v[u].z;
                stage[wave][4 * u + 3][lane] = v[u].w;
            }
            __builtin_amdgcn_wave_barrier();
            // room first: a cut keeps at least k keys and tightens the
            // threshold (the candidates counted above stay a superset)
            if (pool.cnt[0] + total > Pool::CAP) pool.refine(0, k + 128);
            if (pool.cnt[0] + total <= Pool::CAP) {
                // bulk append: this lane's candidates at its prefix position
                int pos = pool.cnt[0] + incl - c;
#pragma unroll 1
                for (int j = 0; c > 0; ++j) {
                    const float x = stage[wave][j][lane];
                    if (score(x) <= th) {
                        const uint32_t i = (uint32_t)(e + (j >> 2) * 256 + lane * 4 + (j & 3));
                        pool_keys[pos++] = make_key(score(x), i);
                        --c;
                    }
                }
                pool.cnt[0] += total;
                appended += total;
                // an offer (up to 64 keys) must find room: cut before it
                pool.need_cut = pool.cnt[0] > Pool::CAP - 64;
            } else {
#pragma unroll 1
                for (int j = 0; j < 4 * U; ++j)
                    offer(stage[wave][j][lane], (uint32_t)(e + (j >> 2) * 256 + lane * 4 + (j & 3)),
                          true);
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll 1
        for (int64_t e = vec_end; e < hi; e += 64) {
            const int64_t i = e + lane;
            offer(i < hi ? rp[i] : 0.f, (uint32_t)i, i < hi);
        }
        // every score at or below the guess was appended (or beaten by k
        // appended ones): with k of them the result is exact
        if (appended >= k || guess == INFINITY) break;
        guess = INFINITY;
    }
    pool.finish();  // at most 64 KR keys left, sentinel padded to that length
    // the pool's appends by every lane are visible to this wave's loads
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    WaveSelect<KR, T> ws;
    ws.init(k);
#pragma unroll 1
    for (int r = 0; r < KR; ++r)
        if (ws.push(pool_keys[r * 64 + lane])) ws.merge();
    ws.finish();
    if (nseg == 1) {
        emit_values<KR, LARGEST>(ws.w, k, vals + row * k, idx + row * k);
    } else {
        emit_keys<KR>(ws.w, k, partial + unit * k);
    }
}

// Pass 2: per row, select the k best of nseg * k partial keys (or, with
// seg_offs, of the lists seg_offs[row] .. seg_offs[row + 1] - 1), written as
// (value, index) pairs or, with keys_out, as the 64*KR-entry sorted key list.
template <int KR, int T, bool LARGEST>
__global__ __launch_bounds__(64 * kWavesPerBlock) void kselect_merge(
    const uint64_t* __restrict__ partial, int64_t nrows, int32_t nseg, int32_t k,
    float* __restrict__ vals, int64_t* __restrict__ idx, uint64_t* __restrict__ keys_out,
    const int64_t* __restrict__ seg_offs) {
    const int wave = threadIdx.x / 64;
    const int lane = lane_id();
    const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (row >= nrows) return;
    const int64_t s0 = seg_offs ? seg_offs[row] : row * (int64_t)nseg;
    const int64_t s1 = seg_offs ? seg_offs[row + 1] : s0 + nseg;
    const uint64_t* p = partial + s0 * k;
    const int64_t n = (s1 - s0) * k;
    WaveSelect<KR, T> ws;
    ws.init(k);
#pragma unroll 1
    for (int64_t e = 0; e < n; e += 64) {
        const int64_t i = e + lane;
        if (ws.push(i < n ? p[i] : kSentinel)) ws.merge();
    }
    ws.finish();
    if (keys_out)
        emit_keys<KR>(ws.w, 64 * KR, keys_out + row * 64 * KR);
    else
        emit_values<KR, LARGEST>(ws.w, k, vals + row * k, idx + row * k);
}

template <int KR, int T, bool LARGEST>
mk_status kselect_launch(const float* a, int64_t nrows, int64_t len, int32_t k, float* vals,
                         int64_t* idx, hipStream_t stream) {
    constexpr int KS = 64 * KR;
    // Enough waves to fill the chip, but segments long enough that the
    // partial keys stay a small fraction of the input.
    int64_t want = ceil_div(8192, nrows > 0 ? nrows : 1);
    int64_t max_by_len = len / (int64_t)(16 * KS > 4096 ? 16 * KS : 4096);
    int64_t nseg = want < max_by_len ? want : max_by_len;
    if (nseg < 1) nseg = 1;
    if (nseg > 4096) nseg = 4096;
    int64_t seg_len = ceil_div(ceil_div(len, nseg), 256) * 256;
    nseg = len > 0 ? ceil_div(len, seg_len) : 1;
    if (seg_len == 0) seg_len = 256;

    Scratch part, pools;
    if (nseg > 1) {
        mk_status st = part.alloc(sizeof(uint64_t) * (size_t)nrows * (size_t)nseg * (size_t)k, stream);
        if (st != MK_OK) return st;
    }
    const int64_t units = nrows * nseg;
    // queues of 256+ entries over segments of at least 16 queue lengths:
    // there most values are rejected and the pool's cuts are rare; short
    // segments (every value a candidate) sort faster in the register queue
    const bool pool = KR >= 4 && seg_len >= 16 * (int64_t)KS;
    {
        ProfScope prof("kselect_pass1", stream);
        if (pool) {
            MK_TRY(pools.alloc(sizeof(uint64_t) * (size_t)units * 2 * KS, stream));
            unsigned long long* drops = nullptr;
            MK_TRY(pool_drop_counter(&drops));
            hipLaunchKernelGGL((kselect_pool<KR, LARGEST>),
                               dim3((unsigned)ceil_div(units, kWavesPerBlock)),
                               dim3(64 * kWavesPerBlock), 0, stream, a, nrows, len, k,
                               (int32_t)nseg, seg_len, vals, idx, part.as<uint64_t>(),
                               pools.as<uint64_t>(), drops);
        } else {
            hipLaunchKernelGGL((kselect_pass1<KR, T, LARGEST>),
                               dim3((unsigned)ceil_div(units, kWavesPerBlock)),
                               dim3(64 * kWavesPerBlock), 0, stream, a, nrows, len, k,
                               (int32_t)nseg, seg_len, vals, idx, part.as<uint64_t>());
        }
        MK_LAUNCHED();
    }
    if (nseg > 1) {
        hipLaunchKernelGGL((kselect_merge<KR, T, LARGEST>),
                           dim3((unsigned)ceil_div(nrows, kWavesPerBlock)), dim3(64 * kWavesPerBlock),
                           0, stream, part.as<uint64_t>(), nrows, (int32_t)nseg, k, vals, idx,
                           (uint64_t*)nullptr, (const int64_t*)nullptr);
        MK_LAUNCHED();
    }
    return MK_OK;
}

template <bool LARGEST>
mk_status kselect_dispatch(const float* a, int64_t nrows, int64_t len, int32_t k, float* vals,
                           int64_t* idx, hipStream_t s) {
    switch (queue_regs(k)) {
        case 1: return kselect_launch<1, SelParams<1>::T, LARGEST>(a, nrows, len, k, vals, idx, s);
        case 2: return kselect_launch<2, SelParams<2>::T, LARGEST>(a, nrows, len, k, vals, idx, s);
        case 4: return kselect_launch<4, SelParams<4>::T, LARGEST>(a, nrows, len, k, vals, idx, s);
        case 8: return kselect_launch<8, SelParams<8>::T, LARGEST>(a, nrows, len, k, vals, idx, s);
        default: return kselect_launch<16, SelParams<16>::T, LARGEST>(a, nrows, len, k, vals, idx, s);
    }
}

}  // namespace

mk_status merge_key_lists(const uint64_t* partial, int64_t nrows, int32_t nseg, int32_t k,
                          float* vals, int64_t* idx, hipStream_t s, uint64_t* keys_out,
                          const int64_t* seg_offs, bool largest) {
    if (nrows == 0) return MK_OK;
    const dim3 grid((unsigned)ceil_div(nrows, kWavesPerBlock)), block(64 * kWavesPerBlock);
    if (largest) {
        MK_REQUIRE(!keys_out, MK_ERR_INVALID_ARG, "largest-first merges emit values");
        switch (queue_regs(k)) {
            case 1: hipLaunchKernelGGL((kselect_merge<1, SelParams<1>::T, true>), grid, block, 0,
                                       s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
            case 2: hipLaunchKernelGGL((kselect_merge<2, SelParams<2>::T, true>), grid, block, 0,
                                       s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
            case 4: hipLaunchKernelGGL((kselect_merge<4, SelParams<4>::T, true>), grid, block, 0,
                                       s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
            case 8: hipLaunchKernelGGL((kselect_merge<8, SelParams<8>::T, true>), grid, block, 0,
                                       s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
            default: hipLaunchKernelGGL((kselect_merge<16, SelParams<16>::T, true>), grid, block, 0,
                                        s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
        }
        MK_LAUNCHED();
        return MK_OK;
    }
    switch (queue_regs(k)) {
        case 1: hipLaunchKernelGGL((kselect_merge<1, SelParams<1>::T, false>), grid, block, 0, s,
                                   partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
        case 2: hipLaunchKernelGGL((kselect_merge<2, SelParams<2>::T, false>), grid, block, 0, s,
                                   partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
        case 4: hipLaunchKernelGGL((kselect_merge<4, SelParams<4>::T, false>), grid, block, 0, s,
                                   partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
        case 8: hipLaunchKernelGGL((kselect_merge<8, SelParams<8>::T, false>), grid, block, 0, s,
                                   partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
        default: hipLaunchKernelGGL((kselect_merge<16, SelParams<16>::T, false>), grid, block, 0,
                                    s, partial, nrows, nseg, k, vals, idx, keys_out, seg_offs); break;
    }
    MK_LAUNCHED();
    return MK_OK;
}

}  // namespace mk

extern "C" mk_status mk_kselect(const float* a, int64_t nrows, int64_t len, int32_t k,
                                int32_t largest, float* vals, int64_t* idx, mk_stream_t stream) {
    MK_REQUIRE(nrows >= 0 && len >= 0, MK_ERR_INVALID_ARG, "nrows and len must be >= 0");
    MK_REQUIRE(k >= 1, MK_ERR_INVALID_ARG, "k must be >= 1");
    MK_REQUIRE(k <= mk::kMaxK, MK_ERR_UNSUPPORTED, "k must be <= 1024");
    MK_REQUIRE(len < (int64_t)0xFFFFFFFF, MK_ERR_UNSUPPORTED, "rows must be shorter than 2^32-1");
    if (nrows == 0) return MK_OK;
    MK_REQUIRE(vals && idx && (a || len == 0), MK_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return largest ? mk::kselect_dispatch<true>(a, nrows, len, k, vals, idx, s)
                   : mk::kselect_dispatch<false>(a, nrows, len, k, vals, idx, s);
}
