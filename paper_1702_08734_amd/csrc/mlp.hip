// Probe-count predictor for IVFADC: a two-hidden-layer ReLU perceptron that
// maps [query ; its 32 smallest squared coarse distances] to log2 of the
// number of inverted lists to probe (an extension of the fixed probe count
// tau of Section 2, Eq. 5).  Forward and backward passes run on the matrix
// cores (FP32 16x16x4 or BF16 16x16x32 MFMA with FP32 accumulation) with the
// master weights, gradients and Adam moments kept in FP32.
//
// Parameters are one flat FP32 vector: W1 [h, din] (row-major), b1 [h],
// W2 [h, h], b2 [h], w3 [h], b3 [1].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "fileio.hpp"
#include "mlp.hpp"
#include "profile.hpp"

struct mk_mlp {
    int32_t din = 0, h = 0;
    mk_precision prec = MK_PREC_FP32;
    int64_t np = 0;
    float* theta = nullptr;    // master parameters
    float* grad = nullptr;     // last gradient
    float* m1 = nullptr;       // Adam first moment
    float* m2 = nullptr;       // Adam second moment
    float* mean = nullptr;     // [din] feature means
    float* inv_std = nullptr;  // [din] 1 / feature standard deviations
    int64_t step = 0;          // Adam steps taken
};

namespace mk {

namespace {

constexpr int kBlock = 256;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct Layout {
    int64_t W1, b1, W2, b2, w3, b3, n;
};

Layout layout(int64_t din, int64_t h) {
    Layout l;
    l.W1 = 0;
    l.b1 = l.W1 + h * din;
    l.W2 = l.b1 + h;
    l.b2 = l.W2 + h * h;
    l.w3 = l.b2 + h;
    l.b3 = l.w3 + h;
    l.n = l.b3 + 1;
    return l;
}

unsigned grid_of(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, kBlock); }

__device__ __forceinline__ uint32_t bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;  // round to nearest even
}

// C[M, N] = op(A) op(B) with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn],
// then + bias[n], relu, and zero where mask[m ldm + n] <= 0 (each optional).
struct GemmArgs {
    const float* A;
    int64_t sam, sak;
    const float* B;
    int64_t sbk, sbn;
    float* C;
    int64_t ldc;
    int32_t M, N, K;
    const float* bias;
    const float* mask;
    int64_t ldm;
    int32_t relu;
};

// 64 x 64 output tile per workgroup, four waves of 2 x 2 blocks of 16 x 16,
// K in steps of 32 staged in LDS.  Lane (i, h) of a block supplies row i of A
// and column i of B for the k-group h; the output element (i, j) of a block
// sits in lane j + 16 (i / 4), element i % 4.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_gemm(GemmArgs g) {
    __shared__ float As[64][33];
    __shared__ float Bs[32][65];
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lh = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += 32) {
        for (int e = tid; e < 64 * 32; e += 256) {
            const int r = e >> 5, c = e & 31;
            const int64_t m = m0 + r, k = k0 + c;
            As[r][c] = (m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.f;
        }
        for (int e = tid; e < 32 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int64_t k = k0 + r, n = n0 + c;
            Bs[r][c] = (k < g.K && n < g.N) ? g.B[k * g.sbk + n * g.sbn] : 0.f;
        }
        __syncthreads();
        if constexpr (BF16) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                uint32_t p[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    p[t] = bf16_bits(As[wm + a * 16 + li][lh * 8 + 2 * t]) |
                           (bf16_bits(As[wm + a * 16 + li][lh * 8 + 2 * t + 1]) << 16);
                av[a] = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                uint32_t p[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    p[t] = bf16_bits(Bs[lh * 8 + 2 * t][wn + b * 16 + li]) |
                           (bf16_bits(Bs[lh * 8 + 2 * t + 1][wn + b * 16 + li]) << 16);
                bv[b] = __builtin_bit_cast(bf16x8, make_uint4(p[0], p[1], p[2], p[3]));
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        } else {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = As[wm + a * 16 + li][kk * 4 + lh];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = Bs[kk * 4 + lh][wn + b * 16 + li];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + a * 16 + 4 * lh + r;
                const int64_t n = n0 + wn + b * 16 + li;
                if (m < g.M && n < g.N) {
                    float v = acc[a][b][r];
                    if (g.bias) v += g.bias[n];
                    if (g.relu) v = fmaxf(v, 0.f);
                    if (g.mask && !(g.mask[m * g.ldm + n] > 0.f)) v = 0.f;
                    g.C[m * g.ldc + n] = v;
                }
            }
}

mk_status gemm(const mk_mlp* net, const GemmArgs& g, hipStream_t s) {
    if (g.M == 0 || g.N == 0) return MK_OK;
    const dim3 grid((unsigned)ceil_div(g.N, 64), (unsigned)ceil_div(g.M, 64));
    if (net->prec == MK_PREC_BF16)
        hipLaunchKernelGGL(mlp_gemm<true>, grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(mlp_gemm<false>, grid, dim3(256), 0, s, g);
    MK_LAUNCHED();
    return MK_OK;
}

GemmArgs gemm_args(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                   int64_t sbn, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K) {
    GemmArgs g{};
    g.A = A; g.sam = sam; g.sak = sak;
    g.B = B; g.sbk = sbk; g.sbn = sbn;
    g.C = C; g.ldc = ldc;
    g.M = (int32_t)M; g.N = (int32_t)N; g.K = (int32_t)K;
    return g;
}

// Xs[i][t] = (F[row i][t] - mean[t]) * inv_std[t], row i = rows ? rows[i] : i.
__global__ void standardize_kernel(const float* __restrict__ F, const int64_t* __restrict__ rows,
                                   int64_t n, int32_t din, const float* __restrict__ mean,
                                   const float* __restrict__ inv_std, float* __restrict__ Xs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * din) return;
    const int64_t i = e / din;
    const int t = (int)(e % din);
    const int64_t r = rows ? rows[i] : i;
    Xs[e] = (F[r * din + t] - mean[t]) * inv_std[t];
}

// yhat[m] = b3 + sum_n H2[m][n] w3[n]; one wave per row, fixed summation order.
__global__ void out_forward_kernel(const float* __restrict__ H2, int64_t n, int32_t h,
                                   const float* __restrict__ w3, const float* __restrict__ b3,
                                   float* __restrict__ yhat) {
    const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (m >= n) return;
    float s = 0.f;
    for (int j = lane; j < h; j += 64) s = fmaf(H2[m * h + j], w3[j], s);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) yhat[m] = s + b3[0];
}

// Residuals of one batch: dy[m] = 2 (yhat[m] - y[m]) / B and the mean squared
// error; a single workgroup, fixed reduction order.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ yhat,
                                                   const float* __restrict__ y,
                                                   const int64_t* __restrict__ rows, int64_t B,
                                                   float* __restrict__ dy,
                                                   float* __restrict__ loss) {
    __shared__ float part[256];
    float s = 0.f;
    for (int64_t m = threadIdx.x; m < B; m += 256) {
        const float r = yhat[m] - y[rows ? rows[m] : m];
        dy[m] = 2.f * r / (float)B;
        s = fmaf(r, r, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = part[0] / (float)B;
}

// dZ2[m][j] = dy[m] w3[j] where H2[m][j] > 0, else 0.
__global__ void out_backward_kernel(const float* __restrict__ dy, const float* __restrict__ w3,
                                    const float* __restrict__ H2, int64_t B, int32_t h,
                                    float* __restrict__ dZ2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * h) return;
    const int64_t m = e / h;
    const int j = (int)(e % h);
    dZ2[e] = H2[e] > 0.f ? dy[m] * w3[j] : 0.f;
}

// out[j] = sum_m wgt[m] X[m][j] (wgt optional).  A workgroup takes 64 columns;
// its 16 row groups each sum every 16th row, then a fixed tree adds the 16
// partial sums (the same order on every call).
constexpr int kColRows = 16;

__global__ __launch_bounds__(64 * kColRows) void colsum_kernel(const float* __restrict__ X,
                                                               int64_t B, int32_t N,
                                                               const float* __restrict__ wgt,
                                                               float* __restrict__ out) {
    __shared__ float part[kColRows][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s = 0.f;
    if (j < N) {
        for (int64_t m = g; m < B; m += kColRows)
            s = wgt ? fmaf(wgt[m], X[m * N + j], s) : s + X[m * N + j];
    }
    part[g][c] = s;
    __syncthreads();
    for (int w = kColRows / 2; w >= 1; w >>= 1) {
        if (g < w) part[g][c] += part[g + w][c];
        __syncthreads();
    }
    if (g == 0 && j < N) out[j] = part[0][c];
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2, int64_t n, float lr,
                            float beta1, float beta2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = beta1 * m1[i] + (1.f - beta1) * gi;
    const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

// Work buffers of one pass over B rows.
struct Pass {
    Scratch xs, h1, h2, yhat, dy, dz2, dz1, loss;
    mk_status alloc(const mk_mlp* net, int64_t B, bool backward, hipStream_t s) {
        MK_TRY(xs.alloc(sizeof(float) * B * net->din, s));
        MK_TRY(h1.alloc(sizeof(float) * B * net->h, s));
        MK_TRY(h2.alloc(sizeof(float) * B * net->h, s));
        MK_TRY(yhat.alloc(sizeof(float) * B, s));
        if (backward) {
            MK_TRY(dy.alloc(sizeof(float) * B, s));
            MK_TRY(dz2.alloc(sizeof(float) * B * net->h, s));
            MK_TRY(dz1.alloc(sizeof(float) * B * net->h, s));
            MK_TRY(loss.alloc(sizeof(float), s));
        }
        return MK_OK;
    }
};

mk_status forward(const mk_mlp* net, const float* F, const int64_t* rows, int64_t B, Pass& p,
                  hipStream_t s) {
    const Layout L = layout(net->din, net->h);
    const int64_t din = net->din, h = net->h;
    hipLaunchKernelGGL(standardize_kernel, dim3(grid_of(B * din)), dim3(kBlock), 0, s, F, rows,
                       B, net->din, net->mean, net->inv_std, p.xs.as<float>());
    MK_LAUNCHED();
    // h1 = relu(Xs W1^T + b1), h2 = relu(h1 W2^T + b2)
    GemmArgs g1 = gemm_args(p.xs.as<float>(), din, 1, net->theta + L.W1, 1, din,
                            p.h1.as<float>(), h, B, h, din);
    g1.bias = net->theta + L.b1;
    g1.relu = 1;
    MK_TRY(gemm(net, g1, s));
    GemmArgs g2 = gemm_args(p.h1.as<float>(), h, 1, net->theta + L.W2, 1, h, p.h2.as<float>(),
                            h, B, h, h);
    g2.bias = net->theta + L.b2;
    g2.relu = 1;
    MK_TRY(gemm(net, g2, s));
    hipLaunchKernelGGL(out_forward_kernel, dim3((unsigned)ceil_div(B * 64, kBlock)), dim3(kBlock),
                       0, s, p.h2.as<float>(), B, net->h, net->theta + L.w3, net->theta + L.b3,
                       p.yhat.as<float>());
    MK_LAUNCHED();
    return MK_OK;
}

// Gradient of the batch's mean squared error into net->grad; loss (device
// scalar) optional.
mk_status backward(mk_mlp* net, const float* y, const int64_t* rows, int64_t B, Pass& p,
                   float* loss, hipStream_t s) {
    const Layout L = layout(net->din, net->h);
    const int64_t din = net->din, h = net->h;
    float* G = net->grad;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, p.yhat.as<float>(), y, rows, B,
                       p.dy.as<float>(), loss ? loss : p.loss.as<float>());
    MK_LAUNCHED();
    hipLaunchKernelGGL(out_backward_kernel, dim3(grid_of(B * h)), dim3(kBlock), 0, s,
                       p.dy.as<float>(), net->theta + L.w3, p.h2.as<float>(), B, net->h,
                       p.dz2.as<float>());
    MK_LAUNCHED();
    // g_w3 = h2^T dy, g_b3 = sum dy, g_b2 = column sums of dz2
    const dim3 cgrid((unsigned)ceil_div(h, 64)), cblock(64 * kColRows);
    hipLaunchKernelGGL(colsum_kernel, cgrid, cblock, 0, s, p.h2.as<float>(), B, net->h,
                       p.dy.as<float>(), G + L.w3);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), cblock, 0, s, p.dy.as<float>(), B, 1,
                       (const float*)nullptr, G + L.b3);
    hipLaunchKernelGGL(colsum_kernel, cgrid, cblock, 0, s, p.dz2.as<float>(), B, net->h,
                       (const float*)nullptr, G + L.b2);
    MK_LAUNCHED();
    // g_W2 = dz2^T h1
    MK_TRY(gemm(net, gemm_args(p.dz2.as<float>(), 1, h, p.h1.as<float>(), h, 1, G + L.W2, h, h, h, B),
                s));
    // dz1 = (dz2 W2) where h1 > 0
    GemmArgs gd = gemm_args(p.dz2.as<float>(), h, 1, net->theta + L.W2, h, 1, p.dz1.as<float>(),
                            h, B, h, h);
    gd.mask = p.h1.as<float>();
    gd.ldm = h;
    MK_TRY(gemm(net, gd, s));
    hipLaunchKernelGGL(colsum_kernel, cgrid, cblock, 0, s, p.dz1.as<float>(), B, net->h,
                       (const float*)nullptr, G + L.b1);
    MK_LAUNCHED();
    // g_W1 = dz1^T Xs
    MK_TRY(gemm(net, gemm_args(p.dz1.as<float>(), 1, h, p.xs.as<float>(), din, 1, G + L.W1, din, h,
                               din, B),
                s));
    return MK_OK;
}

mk_status adam(mk_mlp* net, float lr, hipStream_t s) {
    constexpr double beta1 = 0.9, beta2 = 0.999;
    net->step += 1;
    const float bc1 = (float)(1.0 - std::pow(beta1, (double)net->step));
    const float bc2 = (float)(1.0 - std::pow(beta2, (double)net->step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_of(net->np)), dim3(kBlock), 0, s, net->theta,
                       net->grad, net->m1, net->m2, net->np, lr, (float)beta1, (float)beta2, 1e-8f,
                       bc1, bc2);
    MK_LAUNCHED();
    return MK_OK;
}

void release(mk_mlp* net) {
    for (float** p : {&net->theta, &net->grad, &net->m1, &net->m2, &net->mean, &net->inv_std}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

}  // namespace

int32_t mlp_inputs(const mk_mlp* net) { return net->din; }

mk_status mlp_forward_dev(const mk_mlp* net, const float* F, int64_t n, float* yhat,
                          hipStream_t s) {
    if (n == 0) return MK_OK;
    Pass p;
    MK_TRY(p.alloc(net, n, false, s));
    MK_TRY(forward(net, F, nullptr, n, p, s));
    MK_HIP(hipMemcpyAsync(yhat, p.yhat.ptr, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    return MK_OK;
}

}  // namespace mk

// ---------------------------------------------------------------- C ABI
extern "C" mk_status mk_mlp_create(int32_t din, int32_t hidden, mk_precision prec,
                                   mk_mlp** out) {
    MK_REQUIRE(out, MK_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    MK_REQUIRE(din >= 1 && hidden >= 1, MK_ERR_INVALID_ARG, "need din >= 1 and hidden >= 1");
    MK_REQUIRE(din <= 4096 && hidden <= 4096, MK_ERR_UNSUPPORTED, "din and hidden must be <= 4096");
    MK_REQUIRE(prec == MK_PREC_FP32 || prec == MK_PREC_BF16, MK_ERR_UNSUPPORTED,
               "precision must be FP32 or BF16");
    mk_mlp* net = new mk_mlp;
    net->din = din;
    net->h = hidden;
    net->prec = prec;
    net->np = mk::layout(din, hidden).n;
    const size_t bytes = sizeof(float) * (size_t)net->np;
    hipError_t e = hipSuccess;
    for (float** p : {&net->theta, &net->grad, &net->m1, &net->m2}) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
        if (e == hipSuccess) e = hipMemset(*p, 0, bytes);
    }
    if (e == hipSuccess) e = hipMalloc(&net->mean, sizeof(float) * din);
    if (e == hipSuccess) e = hipMalloc(&net->inv_std, sizeof(float) * din);
    if (e == hipSuccess) {
        std::vector<float> zero(din, 0.f), one(din, 1.f);
        e = hipMemcpy(net->mean, zero.data(), sizeof(float) * din, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(net->inv_std, one.data(), sizeof(float) * din, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        mk::release(net);
        delete net;
        mk::set_error(std::string("mk_mlp_create: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? MK_ERR_OOM : MK_ERR_DEVICE;
    }
    *out = net;
    return MK_OK;
}

extern "C" void mk_mlp_destroy(mk_mlp* net) {
    if (!net) return;
    (void)hipDeviceSynchronize();
    mk::release(net);
    delete net;
}

extern "C" int64_t mk_mlp_num_params(const mk_mlp* net) { return net ? net->np : 0; }

extern "C" mk_status mk_mlp_set_params(mk_mlp* net, const float* theta) {
    MK_REQUIRE(net && theta, MK_ERR_INVALID_ARG, "null pointer");
    const size_t bytes = sizeof(float) * (size_t)net->np;
    MK_HIP(hipDeviceSynchronize());
    MK_HIP(hipMemcpy(net->theta, theta, bytes, hipMemcpyHostToDevice));
    MK_HIP(hipMemset(net->m1, 0, bytes));
    MK_HIP(hipMemset(net->m2, 0, bytes));
    net->step = 0;
    return MK_OK;
}

extern "C" mk_status mk_mlp_get_params(const mk_mlp* net, float* theta, float* grad) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    const size_t bytes = sizeof(float) * (size_t)net->np;
    MK_HIP(hipDeviceSynchronize());
    if (theta) MK_HIP(hipMemcpy(theta, net->theta, bytes, hipMemcpyDeviceToHost));
    if (grad) MK_HIP(hipMemcpy(grad, net->grad, bytes, hipMemcpyDeviceToHost));
    return MK_OK;
}

extern "C" mk_status mk_mlp_fit_standardization(mk_mlp* net, const float* F, int64_t n,
                                                mk_stream_t stream) {
    MK_REQUIRE(net && F, MK_ERR_INVALID_ARG, "null pointer");
    MK_REQUIRE(n >= 1, MK_ERR_INVALID_ARG, "need n >= 1");
    // A one-off preparation step of training, not part of any search: the
    // rows are copied to the host and the statistics summed there in FP64
    // (two passes, rows in order), so the device runs no FP64 arithmetic.
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t din = net->din;
    std::vector<float> h((size_t)n * din);
    MK_HIP(hipMemcpyAsync(h.data(), F, sizeof(float) * h.size(), hipMemcpyDeviceToHost, s));
    MK_HIP(hipStreamSynchronize(s));
    std::vector<double> mu(din, 0.0), var(din, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < din; ++t) mu[t] += (double)h[(size_t)i * din + t];
    for (int32_t t = 0; t < din; ++t) mu[t] /= (double)n;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < din; ++t) {
            const double d = (double)h[(size_t)i * din + t] - mu[t];
            var[t] += d * d;
        }
    std::vector<float> mean(din), inv(din);
    for (int32_t t = 0; t < din; ++t) {
        double sd = std::sqrt(var[t] / (double)n);
        if (sd == 0.0) sd = 1.0;
        mean[t] = (float)mu[t];
        inv[t] = (float)(1.0 / sd);
    }
    MK_HIP(hipMemcpyAsync(net->mean, mean.data(), sizeof(float) * din, hipMemcpyHostToDevice, s));
    MK_HIP(hipMemcpyAsync(net->inv_std, inv.data(), sizeof(float) * din, hipMemcpyHostToDevice,
                          s));
    MK_HIP(hipStreamSynchronize(s));
    return MK_OK;
}

extern "C" mk_status mk_mlp_get_standardization(const mk_mlp* net, float* mean, float* inv_std) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    MK_HIP(hipDeviceSynchronize());
    if (mean) MK_HIP(hipMemcpy(mean, net->mean, sizeof(float) * net->din, hipMemcpyDeviceToHost));
    if (inv_std)
        MK_HIP(hipMemcpy(inv_std, net->inv_std, sizeof(float) * net->din, hipMemcpyDeviceToHost));
    return MK_OK;
}

extern "C" mk_status mk_mlp_forward(const mk_mlp* net, const float* F, int64_t n, float* yhat,
                                    mk_stream_t stream) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    MK_REQUIRE(n >= 0, MK_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return MK_OK;
    MK_REQUIRE(F && yhat, MK_ERR_INVALID_ARG, "null pointer");
    mk::ProfScope prof("mlp_forward", static_cast<hipStream_t>(stream));
    return mk::mlp_forward_dev(net, F, n, yhat, static_cast<hipStream_t>(stream));
}

extern "C" mk_status mk_mlp_loss_grad(mk_mlp* net, const float* F, const int64_t* rows,
                                      int64_t B, const float* y, float* loss,
                                      mk_stream_t stream) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    MK_REQUIRE(B >= 1, MK_ERR_INVALID_ARG, "need B >= 1");
    MK_REQUIRE(F && y, MK_ERR_INVALID_ARG, "null pointer");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    mk::Pass p;
    MK_TRY(p.alloc(net, B, true, s));
    MK_TRY(mk::forward(net, F, rows, B, p, s));
    return mk::backward(net, y, rows, B, p, loss, s);
}

extern "C" mk_status mk_mlp_train_epoch(mk_mlp* net, const float* F, int64_t n, const float* y,
                                        const int64_t* perm, int32_t batch, float lr,
                                        float* losses, mk_stream_t stream) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    MK_REQUIRE(n >= 0 && batch >= 1, MK_ERR_INVALID_ARG, "need n >= 0 and batch >= 1");
    if (n == 0) return MK_OK;
    MK_REQUIRE(F && y && perm, MK_ERR_INVALID_ARG, "null pointer");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    mk::ProfScope prof("mlp_train_epoch", s);
    mk::Pass p;
    MK_TRY(p.alloc(net, std::min<int64_t>(batch, n), true, s));
    int64_t b = 0;
    for (int64_t off = 0; off < n; off += batch, ++b) {
        const int64_t B = std::min<int64_t>(batch, n - off);
        MK_TRY(mk::forward(net, F, perm + off, B, p, s));
        MK_TRY(mk::backward(net, y, perm + off, B, p, losses ? losses + b : nullptr, s));
        MK_TRY(mk::adam(net, lr, s));
    }
    return MK_OK;
}

// ---------------------------------------------------------------- save / load
namespace {
constexpr char kNetMagic[8] = {'M', 'K', 'M', 'L', 'P', '\0', '\0', '\0'};
constexpr uint32_t kNetVersion = 1;
}  // namespace

extern "C" mk_status mk_mlp_shape(const mk_mlp* net, int32_t* din, int32_t* hidden,
                                  int32_t* prec) {
    MK_REQUIRE(net, MK_ERR_INVALID_ARG, "null network");
    if (din) *din = net->din;
    if (hidden) *hidden = net->h;
    if (prec) *prec = (int32_t)net->prec;
    return MK_OK;
}

extern "C" mk_status mk_mlp_save(const mk_mlp* net, const char* path) {
    MK_REQUIRE(net && path, MK_ERR_INVALID_ARG, "null pointer");
    MK_HIP(hipDeviceSynchronize());
    mk::BinFile f(path, "wb");
    MK_REQUIRE(f.ok(), MK_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
    const int32_t prec = (int32_t)net->prec;
    const bool head = f.put(kNetMagic, 8) && f.put_v(kNetVersion) && f.put_v(net->din) &&
                      f.put_v(net->h) && f.put_v(prec) && f.put_v(net->step);
    MK_REQUIRE(head, MK_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
    const size_t pb = sizeof(float) * (size_t)net->np;
    MK_TRY(mk::put_device(f, net->theta, pb));
    MK_TRY(mk::put_device(f, net->m1, pb));
    MK_TRY(mk::put_device(f, net->m2, pb));
    MK_TRY(mk::put_device(f, net->mean, sizeof(float) * (size_t)net->din));
    MK_TRY(mk::put_device(f, net->inv_std, sizeof(float) * (size_t)net->din));
    MK_REQUIRE(f.close(), MK_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
    return MK_OK;
}

extern "C" mk_status mk_mlp_load(const char* path, mk_mlp** out) {
    MK_REQUIRE(path && out, MK_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    mk::BinFile f(path, "rb");
    MK_REQUIRE(f.ok(), MK_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    uint32_t version = 0;
    int32_t din = 0, h = 0, prec = 0;
    int64_t step = 0;
    const bool head = f.get(magic, 8) && f.get_v(version) && f.get_v(din) && f.get_v(h) &&
                      f.get_v(prec) && f.get_v(step);
    MK_REQUIRE(head && std::memcmp(magic, kNetMagic, 8) == 0, MK_ERR_INVALID_ARG,
               std::string(path) + " is not a network file");
    MK_REQUIRE(version == kNetVersion, MK_ERR_UNSUPPORTED,
               std::string(path) + ": unknown network file version");
    MK_REQUIRE(step >= 0, MK_ERR_INVALID_ARG, std::string(path) + ": bad step count");
    mk_mlp* net = nullptr;
    MK_TRY(mk_mlp_create(din, h, (mk_precision)prec, &net));
    const size_t pb = sizeof(float) * (size_t)net->np;
    mk_status st = mk::get_device(f, net->theta, pb);
    if (st == MK_OK) st = mk::get_device(f, net->m1, pb);
    if (st == MK_OK) st = mk::get_device(f, net->m2, pb);
    if (st == MK_OK) st = mk::get_device(f, net->mean, sizeof(float) * (size_t)din);
    if (st == MK_OK) st = mk::get_device(f, net->inv_std, sizeof(float) * (size_t)din);
    if (st == MK_OK && !f.at_end()) {
        mk::set_error(std::string(path) + " has trailing bytes");
        st = MK_ERR_INVALID_ARG;
    }
    if (st != MK_OK) {
        mk_mlp_destroy(net);
        return st;
    }
    net->step = step;
    *out = net;
    return MK_OK;
}
