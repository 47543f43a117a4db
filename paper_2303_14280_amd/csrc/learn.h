// Device code of the learned block screener shared by the screen and training-data kernels:
// the 16 block features and the network 16 -> 64 -> 64 -> 1 (SiLU) evaluated for 16 blocks
// at once per wave64 on the bf16 matrix cores with FP32 accumulation.
#pragma once
#include "snk_internal.h"

namespace snk {
namespace learn {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// nearest bfloat16 (ties to even; one hardware conversion on gfx950): bit pattern, and its
// value as float
__device__ __forceinline__ unsigned bf16_bits(float x)
{
    return (unsigned)(unsigned short)__builtin_bit_cast(short, (__bf16)x);
}
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_bits(x) << 16); }

__device__ __forceinline__ float silu(float z) { return z * __frcp_rn(1.0f + __expf(-z)); }

__device__ __forceinline__ float lg10(double v) { return v > 1e-40 ? (float)log10(v) : -40.0f; }

// log10 c_AB: 0 for A != B, log10(1/2) for A == B
__device__ __forceinline__ float log_cab(const PairFeat& pf) { return pf.cab < 1.0f ? -0.30102999566f : 0.0f; }

__device__ __forceinline__ float box_dist(float x, float y, float z, const BatchGeo& g)
{
    const float ex = fmaxf(fmaxf(g.lo[0] - x, x - g.hi[0]), 0.0f);
    const float ey = fmaxf(fmaxf(g.lo[1] - y, y - g.hi[1]), 0.0f);
    const float ez = fmaxf(fmaxf(g.lo[2] - z, z - g.hi[2]), 0.0f);
    return sqrtf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
}

// Features of block (pair, batch): pair constants, batch geometry, and the batch's F norms
// and bound factors of the two shells, given as log10 (lU = log10 U, lN = log10 N, each
// clamped below at -40).
__device__ __forceinline__ void block_features(const PairFeat& pf, float lp, const BatchGeo& bg, float lUA,
                                               float lUB, float lNA, float lNB, float f[16])
{
    f[0] = pf.la;
    f[1] = pf.lb;
    f[2] = pf.lzA;
    f[3] = pf.lzB;
    f[4] = pf.ab;
    f[5] = pf.lq;
    f[6] = lp;
    f[7] = box_dist(pf.pc[0], pf.pc[1], pf.pc[2], bg);
    f[8] = bg.hd;
    f[9] = box_dist(pf.a[0], pf.a[1], pf.a[2], bg);
    f[10] = box_dist(pf.b[0], pf.b[1], pf.b[2], bg);
    f[11] = bg.lw;
    f[12] = lNA;
    f[13] = lNB;
    f[14] = fmaxf(log_cab(pf) + lUA + lUB, -40.0f);
    const float dx = pf.pc[0] - bg.ctr[0], dy = pf.pc[1] - bg.ctr[1], dz = pf.pc[2] - bg.ctr[2];
    f[15] = sqrtf(dx * dx + dy * dy + dz * dz);
}

// Register image of the network for one lane of a wave64 that evaluates 16 samples.
// Lane (r = lane % 16, g = lane / 16).  Matrix-core operand layout of the 16x16x16 bf16
// product D = A B (checked by the layout probes): lane (r, g) holds A[r][4g..4g+3],
// B[4g..4g+3][r] and D[4g..4g+3][r].  So the samples are the columns, a layer's output
// tile is directly the next layer's B operand, and each lane supplies features 4g..4g+3.
constexpr int kW2Ld = 68;   // LDS row stride (bf16 elements) of W2: 136 B spreads the rows over the banks

struct MlpRegs {
    bf4 w1[4];          // W1[16m + r][4g + e]
    float b3;
};

// The rest of the network in LDS, shared by the workgroup's waves: W2 as bf16 rows of kW2Ld
// elements; biases, W3 (bf16-rounded values) and the feature normalisation and range.
struct MlpShared {
    short w2[64 * kW2Ld];
    float b1[64], b2[64], w3[64];
    float mean[16], istd[16], lo[16], hi[16];
};

__device__ __forceinline__ short bfs(float x) { return (short)bf16_bits(x); }

// Parameters are bf16-rounded on load (weights and biases), as in the inference form of the
// standalone forward kernel.  The whole workgroup fills S; the caller synchronises before
// the first use.
__device__ inline void load_mlp(const float* __restrict__ params, const MlpNorm& nrm, const float* lo,
                                const float* hi, MlpRegs& R, MlpShared& S)
{
    constexpr int OW1 = 0, OB1 = 1024, OW2 = 1088, OB2 = 5184, OW3 = 5248, OB3 = 5312;
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) S.w2[(i >> 6) * kW2Ld + (i & 63)] = bfs(params[OW2 + i]);
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        S.b1[i] = bf16_round(params[OB1 + i]);
        S.b2[i] = bf16_round(params[OB2 + i]);
        S.w3[i] = bf16_round(params[OW3 + i]);
    }
    for (int i = threadIdx.x; i < 16; i += blockDim.x) {
        S.mean[i] = nrm.mean[i];
        S.istd[i] = nrm.inv_std[i];
        S.lo[i] = lo[i];
        S.hi[i] = hi[i];
    }
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    for (int m = 0; m < 4; ++m)
        for (int e = 0; e < 4; ++e) R.w1[m][e] = bfs(params[OW1 + (16 * m + r) * 16 + 4 * g + e]);
    R.b3 = bf16_round(params[OB3]);
}

// x: raw features 4g..4g+3 of sample r.  Returns the network output of sample r in every
// lane that holds sample r (all of the wave's lanes take part).
__device__ inline float mlp_eval16(const MlpRegs& R, const MlpShared& S, const float x[4])
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    bf4 xb;
    for (int e = 0; e < 4; ++e) xb[e] = bfs((x[e] - S.mean[4 * g + e]) * S.istd[4 * g + e]);
    bf4 h1[4];
    for (int m = 0; m < 4; ++m) {
        const f4v b1 = *reinterpret_cast<const f4v*>(S.b1 + 16 * m + 4 * g);
        f4v acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[m], xb, b1, 0, 0, 0);
        for (int e = 0; e < 4; ++e) h1[m][e] = bfs(silu(acc[e]));
    }
    float y = 0.0f;
    for (int m2 = 0; m2 < 4; ++m2) {
        f4v acc = *reinterpret_cast<const f4v*>(S.b2 + 16 * m2 + 4 * g);
        for (int m = 0; m < 4; ++m) {
            const bf4 w = *reinterpret_cast<const bf4*>(S.w2 + (16 * m2 + r) * kW2Ld + 16 * m + 4 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, h1[m], acc, 0, 0, 0);
        }
        const f4v w3 = *reinterpret_cast<const f4v*>(S.w3 + 16 * m2 + 4 * g);
        for (int e = 0; e < 4; ++e) y = fmaf(w3[e], bf16_round(silu(acc[e])), y);
    }
    y += __shfl_xor(y, 16);
    y += __shfl_xor(y, 32);
    return y + R.b3;
}

}  // namespace learn
}  // namespace snk
