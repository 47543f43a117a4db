// The learned block screener's network, 16 -> 64 -> 64 -> 1 with SiLU, on the GPU:
// forward (FP32, or BF16 operands with FP32 accumulation for inference), the fused loss
// and backward pass of the under-prediction-weighted squared error, and Adam.  The layer
// products of the forward and backward passes, and the weight gradients' sums over samples,
// run on the FP32 matrix cores; the parameters (master weights) stay FP32.
// Parameters are FP32, flattened as W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3.
// Inputs are raw features; the kernels standardise them with the stored mean and 1/std.
#include "snk_internal.h"

namespace snk {
namespace {

constexpr int IN = 16, H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NP = OFF_B3 + 1;
static_assert(NP == kMlpParams, "parameter count");

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
// round to the nearest bfloat16 (ties to even) and back
__device__ __forceinline__ float bf16r(float x)
{
    unsigned u = __float_as_uint(x);
    const unsigned lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    return __uint_as_float(u);
}

constexpr int GS = 64;   // samples per workgroup of the forward and gradient kernels
typedef float f4 __attribute__((ext_vector_type(4)));

// acc[nb] += A B over k < K for the wave's 16-row strip: A(i, k) for strip row i, B(k, c) for
// output column c = 16 nb + j.  Operand layout of the 16x16x4 op: lane l supplies A(l % 16,
// l / 16) and B(l / 16, l % 16); acc[nb][e] holds the output at row 4 (l / 16) + e, column
// 16 nb + l % 16.
template <int NB, int K, typename FA, typename FB>
__device__ __forceinline__ void mma_strip(FA A, FB B, f4 (&acc)[NB])
{
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
        const float a = A(li, k0 + lk);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, B(k0 + lk, 16 * nb + li), acc[nb], 0, 0, 0);
    }
}

// Forward pass of GS samples per workgroup of 256 threads: both hidden layers as 64 x 64
// products on the FP32 matrix cores (wave w rows 16 w ..), the output unit per sample.  BF16
// mode rounds parameters, inputs and activations to bfloat16 (products of bfloat16 values are
// exact in FP32, so this is a bfloat16 product with FP32 sums).
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* __restrict__ params, MlpNorm nrm,
                                                      const float* __restrict__ x, int64_t n, float* __restrict__ y)
{
    __shared__ float w1t[IN][H + 1];
    __shared__ float w2t[H][H + 1];
    __shared__ float wb[3 * H + 1];   // b1, b2, w3, b3
    __shared__ float sx[GS][IN];
    __shared__ float sh[GS][H + 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = 16 * wave;
    auto rd = [](float v) { return BF16 ? bf16r(v) : v; };
    for (int e = t; e < H * IN; e += blockDim.x) w1t[e % IN][e / IN] = rd(params[OFF_W1 + e]);
    for (int e = t; e < H * H; e += blockDim.x) w2t[e % H][e / H] = rd(params[OFF_W2 + e]);
    for (int e = t; e < H; e += blockDim.x) {
        wb[e] = rd(params[OFF_B1 + e]);
        wb[H + e] = rd(params[OFF_B2 + e]);
        wb[2 * H + e] = rd(params[OFF_W3 + e]);
    }
    if (t == 0) wb[3 * H] = rd(params[OFF_B3]);
    const int64_t s0 = (int64_t)blockIdx.x * GS;
    for (int e = t; e < GS * IN; e += blockDim.x) {
        const int k = e / IN, j = e % IN;
        sx[k][j] = s0 + k < n ? rd((x[(s0 + k) * IN + j] - nrm.mean[j]) * nrm.inv_std[j]) : 0.0f;
    }
    __syncthreads();
    f4 acc[4] = {};
    mma_strip<4, IN>([&](int i, int k) { return sx[r0 + i][k]; }, [&](int k, int c) { return w1t[k][c]; }, acc);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 16 * nb + li;
            sh[r0 + 4 * lk + e][c] = rd(silu(acc[nb][e] + wb[c]));
        }
    __syncthreads();
    f4 acc2[4] = {};
    mma_strip<4, H>([&](int i, int k) { return sh[r0 + i][k]; }, [&](int k, int c) { return w2t[k][c]; }, acc2);
    __syncthreads();   // every wave has read its rows of h1 before h2 takes their place
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 16 * nb + li;
            sh[r0 + 4 * lk + e][c] = rd(silu(acc2[nb][e] + wb[H + c]));
        }
    __syncthreads();
    if (t < GS && s0 + t < n) {
        float out = wb[3 * H];
        for (int o = 0; o < H; ++o) out = fmaf(wb[2 * H + o], sh[t][o], out);
        y[s0 + t] = out;
    }
}

// One workgroup of 256 threads takes GS = 64 samples.  Every product of the forward and
// backward pass is a 64 x 64 (or 64 x 16) tile on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, operands and sums in FP32, FP32 master weights): wave w owns rows
// 16 w .. 16 w + 15 of each product, operands staged in LDS.  The per-sample steps (bias,
// SiLU and its derivative, the output unit, the loss) run on the vector units in between.  The
// workgroup's partial gradient sums over its samples (fixed order) go to part[block][NP]; the
// loss partial to part[.][NP].
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ params, MlpNorm nrm,
                                                       const float* __restrict__ x, const float* __restrict__ target,
                                                       const float* __restrict__ dyin, int64_t n, float under,
                                                       float* __restrict__ part)
{
    __shared__ float w[NP];
    __shared__ float w1t[IN][H + 1];   // W1 and W2 transposed: the forward products read them
    __shared__ float w2t[H][H + 1];    // along a row of LDS
    __shared__ float sx[GS][IN];
    __shared__ float sh1[GS][H + 1];
    __shared__ float sd1[GS][H + 1];   // SiLU'(z1), then the layer-1 deltas
    __shared__ float sh2[GS][H + 1];
    __shared__ float sd2[GS][H + 1];   // SiLU'(z2), then the layer-2 deltas
    __shared__ float sdy[GS];
    __shared__ float sl[GS];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = 16 * wave;
    for (int i = t; i < NP; i += blockDim.x) w[i] = params[i];
    for (int e = t; e < H * IN; e += blockDim.x) w1t[e % IN][e / IN] = params[OFF_W1 + e];
    for (int e = t; e < H * H; e += blockDim.x) w2t[e % H][e / H] = params[OFF_W2 + e];
    const int64_t s0 = (int64_t)blockIdx.x * GS;
    for (int e = t; e < GS * IN; e += blockDim.x) {
        const int k = e / IN, j = e % IN;
        sx[k][j] = s0 + k < n ? (x[(s0 + k) * IN + j] - nrm.mean[j]) * nrm.inv_std[j] : 0.0f;
    }
    __syncthreads();
    // layer 1: z1 = x W1^T + b1
    {
        f4 acc[4] = {};
        mma_strip<4, IN>([&](int i, int k) { return sx[r0 + i][k]; },
                         [&](int k, int c) { return w1t[k][c]; }, acc);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = r0 + 4 * lk + e, c = 16 * nb + li;
                const float z = acc[nb][e] + w[OFF_B1 + c];
                sh1[i][c] = silu(z);
                sd1[i][c] = dsilu(z);
            }
    }
    __syncthreads();
    // layer 2: z2 = h1 W2^T + b2
    {
        f4 acc[4] = {};
        mma_strip<4, H>([&](int i, int k) { return sh1[r0 + i][k]; },
                        [&](int k, int c) { return w2t[k][c]; }, acc);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = r0 + 4 * lk + e, c = 16 * nb + li;
                const float z = acc[nb][e] + w[OFF_B2 + c];
                sh2[i][c] = silu(z);
                sd2[i][c] = dsilu(z);
            }
    }
    __syncthreads();
    // output and loss per sample: dy = d loss / d y of the asymmetric squared error (loss mode)
    // or the given dy (backward mode)
    if (t < GS) {
        float y = w[OFF_B3];
        for (int o = 0; o < H; ++o) y = fmaf(w[OFF_W3 + o], sh2[t][o], y);
        float dy = 0.0f, l = 0.0f;
        if (s0 + t < n) {
            if (dyin) {
                dy = dyin[s0 + t];
            } else {
                const float tg = target[s0 + t];
                const float c = y < tg ? under : 1.0f;
                dy = 2.0f * c * (y - tg) / (float)n;
                l = c * (y - tg) * (y - tg) / (float)n;
            }
        }
        sdy[t] = dy;
        sl[t] = l;
    }
    __syncthreads();
    // layer-2 deltas d2 = dy w3 SiLU'(z2)
    for (int e = t; e < GS * H; e += blockDim.x) {
        const int k = e / H, o = e % H;
        sd2[k][o] *= sdy[k] * w[OFF_W3 + o];
    }
    __syncthreads();
    // layer-1 deltas d1 = (d2 W2) SiLU'(z1)
    {
        f4 acc[4] = {};
        mma_strip<4, H>([&](int i, int k) { return sd2[r0 + i][k]; },
                        [&](int k, int c) { return w[OFF_W2 + k * H + c]; }, acc);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = r0 + 4 * lk + e, c = 16 * nb + li;
                sd1[i][c] *= acc[nb][e];
            }
    }
    __syncthreads();
    // the workgroup's partial gradients over its samples
    float* out = part + (int64_t)blockIdx.x * (NP + 1);
    {
        // dW2[o][j] = sum_s d2[s][o] h1[s][j], rows o of this wave
        f4 acc[4] = {};
        mma_strip<4, GS>([&](int i, int k) { return sd2[k][r0 + i]; }, [&](int k, int c) { return sh1[k][c]; },
                         acc);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                out[OFF_W2 + (r0 + 4 * lk + e) * H + 16 * nb + li] = acc[nb][e];
        // dW1[o][j] = sum_s d1[s][o] x[s][j]
        f4 acc1[1] = {};
        mma_strip<1, GS>([&](int i, int k) { return sd1[k][r0 + i]; }, [&](int k, int c) { return sx[k][c]; },
                         acc1);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[OFF_W1 + (r0 + 4 * lk + e) * IN + li] = acc1[0][e];
    }
    if (t < H) {
        float g1 = 0.0f, g2 = 0.0f, g3 = 0.0f;
        for (int k = 0; k < GS; ++k) {
            g1 += sd1[k][t];
            g2 += sd2[k][t];
            g3 = fmaf(sdy[k], sh2[k][t], g3);
        }
        out[OFF_B1 + t] = g1;
        out[OFF_B2 + t] = g2;
        out[OFF_W3 + t] = g3;
    } else if (t == H) {
        float g = 0.0f, l = 0.0f;
        for (int k = 0; k < GS; ++k) {
            g += sdy[k];
            l += sl[k];
        }
        out[OFF_B3] = g;
        out[NP] = l;
    }
}

// grads[p] = sum over blocks of part[b][p] (fixed order); loss in grads[NP]
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ grads)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += part[(int64_t)b * (NP + 1) + p];
    grads[p] = g;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ params, float* __restrict__ m,
                                                       float* __restrict__ v, const float* __restrict__ g, float lr,
                                                       float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float gi = g[p];
    const float mi = 0.9f * m[p] + 0.1f * gi;
    const float vi = 0.999f * v[p] + 0.001f * gi * gi;
    m[p] = mi;
    v[p] = vi;
    params[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

}  // namespace

hipError_t launch_mlp_forward(const float* params, const MlpNorm& nrm, const float* x, int64_t n, float* y, bool bf16,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + GS - 1) / GS)), block(256);
    if (bf16)
        hipLaunchKernelGGL((mlp_fwd_kernel<true>), grid, block, 0, s, params, nrm, x, n, y);
    else
        hipLaunchKernelGGL((mlp_fwd_kernel<false>), grid, block, 0, s, params, nrm, x, n, y);
    return hipGetLastError();
}

int64_t mlp_grad_blocks(int64_t n) { return (n + GS - 1) / GS; }

namespace {
__global__ __launch_bounds__(256) void log10_kernel(const double* __restrict__ in, int64_t n, float* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] > 1e-40 ? (float)log10(in[i]) : -40.0f;
}
}  // namespace

hipError_t launch_log10(const double* in, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(log10_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const MlpNorm& nrm, const float* x, const float* target,
                           const float* dy, int64_t n, float under, float* part, float* grads, hipStream_t s)
{
    const int64_t nblk = mlp_grad_blocks(n);
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)nblk), dim3(256), 0, s, params, nrm, x, target, dy, n, under,
                       part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, part, (int)nblk, grads);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* g, float lr, int t, hipStream_t s)
{
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, params, m, v, g, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace snk
