// The learned block screener's network, 16 -> 64 -> 64 -> 1 with SiLU, on the GPU:
// forward (FP32, or BF16 operands with FP32 accumulation for inference), the fused loss
// and backward pass of the under-prediction-weighted squared error, and Adam.
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

template <bool BF16>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* __restrict__ params, MlpNorm nrm,
                                                      const float* __restrict__ x, int64_t n, float* __restrict__ y)
{
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = BF16 ? bf16r(params[i]) : params[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xi[IN];
    for (int j = 0; j < IN; ++j) {
        const float v = (x[s * IN + j] - nrm.mean[j]) * nrm.inv_std[j];
        xi[j] = BF16 ? bf16r(v) : v;
    }
    float h1[H];
    for (int o = 0; o < H; ++o) {
        float z = w[OFF_B1 + o];
        for (int j = 0; j < IN; ++j) z = fmaf(w[OFF_W1 + o * IN + j], xi[j], z);
        h1[o] = BF16 ? bf16r(silu(z)) : silu(z);
    }
    float out = w[OFF_B3];
    for (int o = 0; o < H; ++o) {
        float z = w[OFF_B2 + o];
        for (int j = 0; j < H; ++j) z = fmaf(w[OFF_W2 + o * H + j], h1[j], z);
        const float h2 = BF16 ? bf16r(silu(z)) : silu(z);
        out = fmaf(w[OFF_W3 + o], h2, out);
    }
    y[s] = out;
}

// One workgroup of 256 threads takes 64 samples: threads 0..63 run the forward and backward
// pass of one sample each into LDS, then all threads form the workgroup's partial gradient
// sums over its samples (fixed order), written to part[block][NP]; loss partial in part[.][NP].
constexpr int GS = 64;
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ params, MlpNorm nrm,
                                                       const float* __restrict__ x, const float* __restrict__ target,
                                                       const float* __restrict__ dyin, int64_t n, float under,
                                                       float* __restrict__ part)
{
    __shared__ float w[NP];
    __shared__ float sx[GS][IN];
    __shared__ float sh1[GS][H];
    __shared__ float sh2[GS][H];
    __shared__ float sd1[GS][H];
    __shared__ float sd2[GS][H];
    __shared__ float sdy[GS];
    __shared__ float sl[GS];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = params[i];
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * GS + t;
    if (t < GS) {
        float xi[IN];
        float z1[H], h1[H], z2[H];
        const bool live = s < n;
        for (int j = 0; j < IN; ++j) {
            xi[j] = live ? (x[s * IN + j] - nrm.mean[j]) * nrm.inv_std[j] : 0.0f;
            sx[t][j] = xi[j];
        }
        for (int o = 0; o < H; ++o) {
            float z = w[OFF_B1 + o];
            for (int j = 0; j < IN; ++j) z = fmaf(w[OFF_W1 + o * IN + j], xi[j], z);
            z1[o] = z;
            h1[o] = silu(z);
            sh1[t][o] = h1[o];
        }
        float y = w[OFF_B3];
        for (int o = 0; o < H; ++o) {
            float z = w[OFF_B2 + o];
            for (int j = 0; j < H; ++j) z = fmaf(w[OFF_W2 + o * H + j], h1[j], z);
            z2[o] = z;
            const float h2 = silu(z);
            sh2[t][o] = h2;
            y = fmaf(w[OFF_W3 + o], h2, y);
        }
        // loss mode: dy = d loss / d y of the asymmetric squared error; backward mode: dy given
        float dy = 0.0f, l = 0.0f;
        if (live) {
            if (dyin) {
                dy = dyin[s];
            } else {
                const float tg = target[s];
                const float c = y < tg ? under : 1.0f;
                dy = 2.0f * c * (y - tg) / (float)n;
                l = c * (y - tg) * (y - tg) / (float)n;
            }
        }
        sdy[t] = dy;
        sl[t] = l;
        float d2[H];
        for (int o = 0; o < H; ++o) {
            d2[o] = dy * w[OFF_W3 + o] * dsilu(z2[o]);
            sd2[t][o] = d2[o];
        }
        for (int j = 0; j < H; ++j) {
            float a = 0.0f;
            for (int o = 0; o < H; ++o) a = fmaf(d2[o], w[OFF_W2 + o * H + j], a);
            sd1[t][j] = a * dsilu(z1[j]);
        }
    }
    __syncthreads();
    float* out = part + (int64_t)blockIdx.x * (NP + 1);
    for (int p = t; p < NP; p += blockDim.x) {
        float g = 0.0f;
        if (p < OFF_B1) {
            const int o = (p - OFF_W1) / IN, j = (p - OFF_W1) % IN;
            for (int k = 0; k < GS; ++k) g = fmaf(sd1[k][o], sx[k][j], g);
        } else if (p < OFF_W2) {
            const int o = p - OFF_B1;
            for (int k = 0; k < GS; ++k) g += sd1[k][o];
        } else if (p < OFF_B2) {
            const int o = (p - OFF_W2) / H, j = (p - OFF_W2) % H;
            for (int k = 0; k < GS; ++k) g = fmaf(sd2[k][o], sh1[k][j], g);
        } else if (p < OFF_W3) {
            const int o = p - OFF_B2;
            for (int k = 0; k < GS; ++k) g += sd2[k][o];
        } else if (p < OFF_B3) {
            const int o = p - OFF_W3;
            for (int k = 0; k < GS; ++k) g = fmaf(sdy[k], sh2[k][o], g);
        } else {
            for (int k = 0; k < GS; ++k) g += sdy[k];
        }
        out[p] = g;
    }
    if (t == 0) {
        float l = 0.0f;
        for (int k = 0; k < GS; ++k) l += sl[k];
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
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
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
