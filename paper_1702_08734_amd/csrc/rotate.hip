// Linear pre-processing of rows (an OPQ rotation or a projection, Sections 1
// and 6.4): out[i][j] = sum_t x[i][t] * rot[j][t] on the FP32 matrix cores.
//
// One workgroup per 64 x 64 output tile, four waves of 2 x 2 blocks of
// 16 x 16 (v_mfma_f32_16x16x4f32).  K goes in chunks of 32 staged whole in
// LDS (rows of x and of rot, both K-contiguous, one barrier pair per chunk);
// LDS rows are 34 floats apart so that the operand reads of a 32-lane half
// (16 rows x 2 k-groups) fall in 32 distinct banks.  The 17 KB of LDS per
// workgroup let the CU hold as many workgroups as its wave slots allow, and
// their staging overlaps each other's matrix work (chunks of 64, 34 KB:
// 4.9 ms for 10^7 x 128 rows; chunks of 32: 4.0 ms).  Consecutive workgroups
// share a row tile (its loads hit L2).  Every output element sums its
// products in one fixed order, so the result is deterministic.
#include "common.hpp"

namespace mk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // rows and columns of an output tile
constexpr int kKC = 32;     // K per LDS stage
constexpr int kLds = kKC + 2;

// Rows [r0, r0 + 64) x k [k0, k0 + 32) of a row-major [rows, d] matrix into
// S (zero outside), 256 threads; float4 loads when vec.
__device__ __forceinline__ void stage(float (*S)[kLds], const float* __restrict__ m, int64_t rows,
                                      int32_t d, int64_t r0, int32_t k0, bool vec) {
    const int tid = threadIdx.x;
    if (vec) {
#pragma unroll
        for (int e = tid; e < kTile * (kKC / 4); e += 256) {
            const int r = e / (kKC / 4), c = 4 * (e % (kKC / 4));
            const int64_t row = r0 + r;
            const int32_t k = k0 + c;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (row < rows && k < d) v = *reinterpret_cast<const float4*>(m + row * d + k);
            *reinterpret_cast<float2*>(&S[r][c]) = make_float2(v.x, v.y);
            *reinterpret_cast<float2*>(&S[r][c + 2]) = make_float2(v.z, v.w);
        }
    } else {
        for (int e = tid; e < kTile * kKC; e += 256) {
            const int r = e / kKC, c = e % kKC;
            const int64_t row = r0 + r;
            const int32_t k = k0 + c;
            S[r][c] = (row < rows && k < d) ? m[row * d + k] : 0.f;
        }
    }
}

__global__ __launch_bounds__(256) void rotate_rows_kernel(const float* __restrict__ x, int64_t n,
                                                          int32_t d, const float* __restrict__ rot,
                                                          int32_t dout, float* __restrict__ out,
                                                          int64_t ncb, int32_t vec) {
    __shared__ __align__(16) float As[kTile][kLds];
    __shared__ __align__(16) float Bs[kTile][kLds];
    const int64_t b = blockIdx.x;
    const int64_t r0 = (b / ncb) * kTile, c0 = (b % ncb) * kTile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lh = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int32_t k0 = 0; k0 < d; k0 += kKC) {
        if (k0 > 0) __syncthreads();  // the previous chunk's reads are done
        stage(As, x, n, d, r0, k0, vec != 0);
        stage(Bs, rot, dout, d, c0, k0, vec != 0);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKC / 4; ++kk) {
            float av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[wm + i * 16 + li][kk * 4 + lh];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[wn + j * 16 + li][kk * 4 + lh];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i / 4), element i % 4
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + wm + i * 16 + 4 * lh + r;
                const int64_t col = c0 + wn + j * 16 + li;
                if (row < n && col < dout) out[row * dout + col] = acc[i][j][r];
            }
}

}  // namespace
}  // namespace mk

extern "C" mk_status mk_rotate_rows(const float* x, int64_t n, int32_t d, const float* rot,
                                    int32_t dout, float* out, mk_stream_t stream) {
    MK_REQUIRE(n >= 0 && d >= 1 && dout >= 1, MK_ERR_INVALID_ARG, "need n >= 0, d >= 1, dout >= 1");
    if (n == 0) return MK_OK;
    MK_REQUIRE(x && rot && out, MK_ERR_INVALID_ARG, "null pointer");
    const char* xe = reinterpret_cast<const char*>(x + n * (int64_t)d);
    const char* oe = reinterpret_cast<const char*>(out + n * (int64_t)dout);
    MK_REQUIRE(xe <= reinterpret_cast<const char*>(out) || oe <= reinterpret_cast<const char*>(x),
               MK_ERR_INVALID_ARG, "out must not overlap x");
    const int64_t ncb = mk::ceil_div(dout, mk::kTile);
    const int64_t blocks = mk::ceil_div(n, mk::kTile) * ncb;
    MK_REQUIRE(blocks < ((int64_t)1 << 32), MK_ERR_UNSUPPORTED, "too many rows for one call");
    const bool vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(rot) % 16 == 0;
    hipLaunchKernelGGL(mk::rotate_rows_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, n, d, rot, dout, out, ncb,
                       (int32_t)vec);
    MK_LAUNCHED();
    return MK_OK;
}
