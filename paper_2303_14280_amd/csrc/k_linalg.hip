// Dense linear-algebra steps of the sn-K build on gfx950:
//  - FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64) for F = P_g Phi_g (Eq. fmat)
//    and Kt_g = G_g Phi_g^T (Eq. usym_k, split over the grid-point dimension);
//  - deterministic reduction of the split partials into Kt;
//  - K = (Kt + Kt^T)/2 (Eq. sn_k) and E_x = -1/2 tr(P K) by a fixed two-stage tree;
//  - fill and gather helpers.
#include "snk_internal.h"

#include <type_traits>

namespace snk {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int kFlush = 1024;   // FP32 mode: k per FP32 accumulation before the FP64 add

// 256 threads = 4 wave64; wave w owns the 32x32 quadrant (w/2, w%2) of the 64x64 tile as
// 2x2 matrix-core 16x16 blocks.  F32 = false: v_mfma_f64_16x16x4f64, operands and
// accumulators FP64; F32 = true: v_mfma_f32_16x16x4f32, operands rounded to FP32 as they are
// staged (whatever the storage type) and FP32 accumulation.  Operand layout (wave64):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
//   FP64 accumulator D[i][j] in lane j + 16(i%4), element i/4;
//   FP32 accumulator D[i][j] in lane j + 16(i/4), element i%4
// (both accumulator layouts are checked by GEMM tests against host products).
template <typename TA, typename TB, typename TC, bool F32>
__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                   int64_t lda, const TB* __restrict__ B, int64_t ldb, int bt,
                                                   TC* __restrict__ C, int64_t ldc, int64_t kchunk,
                                                   int64_t split_stride)
{
    typedef typename std::conditional<F32, float, double>::type TS;
    typedef TS acc4 __attribute__((ext_vector_type(4)));
    __shared__ TS As[TK][TM + 1];
    __shared__ TS Bs[TK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = min(K, kbeg + kchunk);
    C += (int64_t)blockIdx.z * split_stride;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;

    acc4 acc[2][2];
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc4{0, 0, 0, 0};
    // FP32 mode: the matrix-core accumulators cover at most kFlush consecutive k; they are
    // then added into FP64 accumulators (FP32 sums stay short, long sums are FP64)
    double dacc[2][2][4];
    if constexpr (F32)
        for (int bi = 0; bi < 2; ++bi)
            for (int bj = 0; bj < 2; ++bj)
                for (int r = 0; r < 4; ++r) dacc[bi][bj][r] = 0.0;
    auto flush = [&]() {
        if constexpr (F32)
            for (int bi = 0; bi < 2; ++bi)
                for (int bj = 0; bj < 2; ++bj) {
                    for (int r = 0; r < 4; ++r) dacc[bi][bj][r] += (double)acc[bi][bj][r];
                    acc[bi][bj] = acc4{0, 0, 0, 0};
                }
    };

    const int ai = tid >> 2, ak = (tid & 3) * 4;
    int since_flush = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
        if (F32 && since_flush == kFlush / TK) {
            flush();
            since_flush = 0;
        }
        ++since_flush;
        {
            const int64_t gm = m0 + ai;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t gk = k0 + ak + u;
                As[ak + u][ai] = (gm < M && gk < kend) ? (TS)A[gm * lda + gk] : (TS)0;
            }
        }
        if (!bt) {
            const int bk = tid >> 4, bj = (tid & 15) * 4;
            const int64_t gk = k0 + bk;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t gn = n0 + bj + u;
                Bs[bk][bj + u] = (gk < kend && gn < N) ? (TS)B[gk * ldb + gn] : (TS)0;
            }
        } else {
            const int bj = tid >> 2, bk = (tid & 3) * 4;
            const int64_t gn = n0 + bj;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t gk = k0 + bk + u;
                Bs[bk + u][bj] = (gn < N && gk < kend) ? (TS)B[gn * ldb + gk] : (TS)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            TS a[2], b[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) a[bi] = As[ks + lk][wm + bi * 16 + li];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[ks + lk][wn + bj * 16 + li];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    if constexpr (F32)
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
                    else
                        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    flush();
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm + bi * 16 + (F32 ? 4 * lk + r : 4 * r + lk);
                const int64_t gn = n0 + wn + bj * 16 + li;
                if constexpr (F32) {
                    if (gm < M && gn < N) C[gm * ldc + gn] = (TC)dacc[bi][bj][r];
                } else {
                    if (gm < M && gn < N) C[gm * ldc + gn] = (TC)acc[bi][bj][r];
                }
            }
}

// Row-wise element kernels: blockIdx.y strides the rows, the x blocks of 256 threads stride a
// row's columns (no integer division per element).
#define SNK_ROWS(m, M) for (int64_t m = blockIdx.y; m < (M); m += gridDim.y)
#define SNK_COLS(n, N) \
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < (N); n += (int64_t)gridDim.x * blockDim.x)

dim3 rows_grid(int64_t rows, int64_t cols)
{
    const int64_t gx = std::min<int64_t>(std::max<int64_t>(1, (cols + 255) / 256), 16);
    const int64_t gy = std::min<int64_t>(std::max<int64_t>(1, rows), 65535);
    return dim3((unsigned)gx, (unsigned)gy);
}

template <typename TP>
__global__ __launch_bounds__(256) void reduce_scatter_kernel(const TP* __restrict__ part, int nsplit,
                                                             int64_t stride, int64_t M, int64_t N,
                                                             const int32_t* __restrict__ rows,
                                                             const int32_t* __restrict__ cols,
                                                             double* __restrict__ Kt, int64_t nbf)
{
    SNK_ROWS(m, M)
    {
        double* krow = Kt + (int64_t)(rows ? rows[m] : m) * nbf;
        SNK_COLS(n, N)
        {
            const int64_t idx = m * N + n;
            double s = 0.0;
            for (int z = 0; z < nsplit; ++z) s += (double)part[z * stride + idx];
            krow[cols ? cols[n] : n] += s;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// p[r * ld + c] = v for r < rows, c < cols
template <typename T>
__global__ __launch_bounds__(256) void fill2d_kernel(T* __restrict__ p, int64_t rows, int64_t cols, int64_t ld, T v)
{
    SNK_ROWS(r, rows)
    {
        SNK_COLS(c, cols) p[r * ld + c] = v;
    }
}

__global__ __launch_bounds__(256) void convert_kernel(const double* __restrict__ in, int64_t n, float* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__device__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(256) void finish_kernel(const double* __restrict__ Kt, const double* __restrict__ P,
                                                     double* __restrict__ K, int64_t nbf, double* __restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t n2 = nbf * nbf;
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n2; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / nbf, j = idx - i * nbf;
        const double k = 0.5 * (Kt[idx] + Kt[j * nbf + i]);
        K[idx] = k;
        acc = fma(P[idx], k, acc);   // tr(PK) = sum_ij P_ij K_ji and K is symmetric
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void finish_reduce_kernel(const double* __restrict__ partial, int nblk,
                                                            double* __restrict__ ex)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) ex[0] = -0.5 * s;
}

template <typename TO>
__global__ __launch_bounds__(256) void gather_kernel(const double* __restrict__ P, int64_t nbf,
                                                     const int32_t* __restrict__ rows, int64_t M,
                                                     const int32_t* __restrict__ cols, int64_t N,
                                                     TO* __restrict__ out)
{
    SNK_ROWS(m, M)
    {
        const double* src = P + (int64_t)(rows ? rows[m] : m) * nbf;
        TO* dst = out + m * N;
        SNK_COLS(n, N) dst[n] = (TO)src[cols ? cols[n] : n];
    }
}

// out[rows[m] * ld + c] = in[m * ncols + c]
template <typename T>
__global__ __launch_bounds__(256) void scatter_rows_kernel(const T* __restrict__ in, int64_t M, int64_t ncols,
                                                           const int32_t* __restrict__ rows, T* __restrict__ out,
                                                           int64_t ld)
{
    SNK_ROWS(m, M)
    {
        const T* src = in + m * ncols;
        T* dst = out + (int64_t)rows[m] * ld;
        SNK_COLS(c, ncols) dst[c] = src[c];
    }
}

// p[rows[m] * ld + c] = v for m < M, c < ncols
__global__ __launch_bounds__(256) void fill_rows_kernel(double* __restrict__ p, int64_t ld,
                                                        const int32_t* __restrict__ rows, int64_t M, int64_t ncols,
                                                        double v)
{
    SNK_ROWS(m, M)
    {
        double* dst = p + (int64_t)rows[m] * ld;
        SNK_COLS(c, ncols) dst[c] = v;
    }
}

// One wave per row of a group's Phi buffer (the tiles' Phi_t one after the other: nfull rows
// of ncols_full columns, then the rows of the last tile with ncols_last columns):
// mx[r] = max_c |Phi_r,c|
template <typename T>
__global__ __launch_bounds__(256) void row_absmax_kernel(const T* __restrict__ Phi, int64_t nfull, int64_t ncols_full,
                                                         int64_t nrow, int64_t ncols_last, double* __restrict__ mx)
{
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= nrow) return;
    const bool full = r < nfull;
    const int64_t ncols = full ? ncols_full : ncols_last;
    const T* row = Phi + (full ? r * ncols_full : nfull * ncols_full + (r - nfull) * ncols_last);
    double m = 0.0;
    for (int64_t c = lane; c < ncols; c += 64) m = fmax(m, fabs((double)row[c]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (lane == 0) mx[r] = m;
}

// One wave per (function lam, tile t): Ft = sum_k |P[lam][fn[k]]| mx[k] over the tile's
// functions (rows roff[t] .. roff[t+1]-1 of fn and mx) bounds |F_lam,i| on every point of the
// tile (Eq. fmat with |Phi_nu,i| <= mx); flag[t][shell_of[lam]] = 1 when Ft >= eps.
__global__ __launch_bounds__(256) void ftilde_flag_kernel(const double* __restrict__ P, int64_t nbf,
                                                          const int32_t* __restrict__ fn,
                                                          const int32_t* __restrict__ roff,
                                                          const double* __restrict__ mx, double eps,
                                                          const int32_t* __restrict__ shell_of, int32_t nshell,
                                                          int32_t* __restrict__ flag)
{
    const int64_t lam = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63;
    if (lam >= nbf) return;
    const double* row = P + lam * nbf;
    const int k0 = roff[t], k1 = roff[t + 1];
    double v = 0.0;
    for (int k = k0 + lane; k < k1; k += 64) v = fma(fabs(row[fn[k]]), mx[k], v);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0 && v >= eps) flag[(int64_t)t * nshell + shell_of[lam]] = 1;
}

// One wave: A[i][k] = (k == 0) + i (k == 1), B[k][j] = 100 j (k == 0) + (k == 1), so that
// D[i][j] = 100 j + i; every lane writes its four accumulator elements.
__global__ void mfma_probe_kernel(double* __restrict__ out)
{
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    const double a = k == 0 ? 1.0 : (k == 1 ? (double)i : 0.0);
    const double b = k == 0 ? 100.0 * i : (k == 1 ? 1.0 : 0.0);
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[4 * lane + r] = acc[r];
}

}  // namespace

hipError_t launch_mfma_probe(double* out_dev, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, out_dev);
    return hipGetLastError();
}

namespace {

template <typename TA, typename TB, typename TC, bool F32>
hipError_t launch_gemm_t(int64_t M, int64_t N, int64_t K, const TA* A, int64_t lda, const TB* B, int64_t ldb, bool bt,
                         TC* C, int64_t ldc, int nsplit, int64_t split_stride, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (nsplit < 1) nsplit = 1;
    int64_t kchunk = (K + nsplit - 1) / nsplit;
    kchunk = ((kchunk + TK - 1) / TK) * TK;
    if (kchunk <= 0) kchunk = TK;
    const int64_t nz = (K + kchunk - 1) / kchunk;
    dim3 grid((unsigned)((N + TN - 1) / TN), (unsigned)((M + TM - 1) / TM), (unsigned)(nz > 0 ? nz : 1)), block(256);
    hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, F32>), grid, block, 0, s, M, N, K, A, lda, B, ldb, bt ? 1 : 0, C, ldc,
                       kchunk, split_stride);
    if (nz < nsplit) {
        // chunks beyond the K range would be left unwritten: clear them
        for (int64_t z = nz; z < nsplit; ++z) {
            const int64_t n = M * ldc;
            int64_t blocks = (n + 255) / 256;
            if (blocks > 65536) blocks = 65536;
            hipLaunchKernelGGL((fill_kernel<TC>), dim3((unsigned)blocks), dim3(256), 0, s, C + z * split_stride, n,
                               (TC)0);
        }
    }
    return hipGetLastError();
}

template <typename TP>
hipError_t launch_reduce_scatter_t(const TP* part, int nsplit, int64_t stride, int64_t M, int64_t N,
                                   const int32_t* rows, const int32_t* cols, double* Kt, int64_t nbf, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL((reduce_scatter_kernel<TP>), rows_grid(M, N), dim3(256), 0, s, part, nsplit, stride, M, N, rows,
                       cols, Kt, nbf);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
                           bool bt, double* C, int64_t ldc, int nsplit, int64_t split_stride, hipStream_t s)
{
    return launch_gemm_t<double, double, double, false>(M, N, K, A, lda, B, ldb, bt, C, ldc, nsplit, split_stride, s);
}

hipError_t launch_gemm_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B, int64_t ldb,
                           bool bt, float* C, int64_t ldc, int nsplit, int64_t split_stride, hipStream_t s)
{
    return launch_gemm_t<float, float, float, true>(M, N, K, A, lda, B, ldb, bt, C, ldc, nsplit, split_stride, s);
}

hipError_t launch_gemm_f32_dA(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const float* B,
                              int64_t ldb, bool bt, double* C, int64_t ldc, int nsplit, int64_t split_stride,
                              hipStream_t s)
{
    return launch_gemm_t<double, float, double, true>(M, N, K, A, lda, B, ldb, bt, C, ldc, nsplit, split_stride, s);
}

hipError_t launch_reduce_scatter(const double* part, int nsplit, int64_t stride, int64_t M, int64_t N,
                                 const int32_t* rows, const int32_t* cols, double* Kt, int64_t nbf, hipStream_t s)
{
    return launch_reduce_scatter_t<double>(part, nsplit, stride, M, N, rows, cols, Kt, nbf, s);
}

hipError_t launch_convert_f32(const double* in, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((fill_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fill2d_t(T* p, int64_t rows, int64_t cols, int64_t ld, T v, hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL((fill2d_kernel<T>), rows_grid(rows, cols), dim3(256), 0, s, p, rows, cols, ld, v);
    return hipGetLastError();
}

hipError_t launch_fill2d(double* p, int64_t rows, int64_t cols, int64_t ld, double v, hipStream_t s)
{
    return launch_fill2d_t<double>(p, rows, cols, ld, v, s);
}

hipError_t launch_fill2d(float* p, int64_t rows, int64_t cols, int64_t ld, float v, hipStream_t s)
{
    return launch_fill2d_t<float>(p, rows, cols, ld, v, s);
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((fill_kernel<int32_t>), dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((fill_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_finish(const double* Kt, const double* P, double* K, int64_t nbf, double* partial, int nblk,
                         double* ex, hipStream_t s)
{
    hipLaunchKernelGGL(finish_kernel, dim3(nblk), dim3(256), 0, s, Kt, P, K, nbf, partial);
    hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(256), 0, s, partial, nblk, ex);
    return hipGetLastError();
}

template <typename TO>
static hipError_t launch_gather_t(const double* P, int64_t nbf, const int32_t* rows, int64_t M, const int32_t* cols,
                                  int64_t N, TO* out, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL((gather_kernel<TO>), rows_grid(M, N), dim3(256), 0, s, P, nbf, rows, M, cols, N, out);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_scatter_rows_t(const T* in, int64_t M, int64_t ncols, const int32_t* rows, T* out, int64_t ld,
                                       hipStream_t s)
{
    if (M <= 0 || ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL((scatter_rows_kernel<T>), rows_grid(M, ncols), dim3(256), 0, s, in, M, ncols, rows, out, ld);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(const double* in, int64_t M, int64_t ncols, const int32_t* rows, double* out, int64_t ld,
                               hipStream_t s)
{
    return launch_scatter_rows_t<double>(in, M, ncols, rows, out, ld, s);
}

hipError_t launch_scatter_rows(const float* in, int64_t M, int64_t ncols, const int32_t* rows, float* out, int64_t ld,
                               hipStream_t s)
{
    return launch_scatter_rows_t<float>(in, M, ncols, rows, out, ld, s);
}

hipError_t launch_fill_rows(double* p, int64_t ld, const int32_t* rows, int64_t M, int64_t ncols, double v,
                            hipStream_t s)
{
    if (M <= 0 || ncols <= 0) return hipSuccess;
    if (!p || !rows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_rows_kernel, rows_grid(M, ncols), dim3(256), 0, s, p, ld, rows, M, ncols, v);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_row_absmax_t(const T* Phi, int64_t nfull, int64_t ncols_full, int64_t nrow, int64_t ncols_last,
                                      double* mx, hipStream_t s)
{
    if (nrow <= 0) return hipSuccess;
    if (!Phi || !mx || nfull > nrow) return hipErrorInvalidValue;
    hipLaunchKernelGGL((row_absmax_kernel<T>), dim3((unsigned)((nrow + 3) / 4)), dim3(256), 0, s, Phi, nfull,
                       ncols_full, nrow, ncols_last, mx);
    return hipGetLastError();
}

hipError_t launch_row_absmax(const double* Phi, int64_t nfull, int64_t ncols_full, int64_t nrow, int64_t ncols_last,
                             double* mx, hipStream_t s)
{
    return launch_row_absmax_t<double>(Phi, nfull, ncols_full, nrow, ncols_last, mx, s);
}

hipError_t launch_row_absmax(const float* Phi, int64_t nfull, int64_t ncols_full, int64_t nrow, int64_t ncols_last,
                             double* mx, hipStream_t s)
{
    return launch_row_absmax_t<float>(Phi, nfull, ncols_full, nrow, ncols_last, mx, s);
}

hipError_t launch_ftilde_flag(const double* P, int64_t nbf, const int32_t* fn, const int32_t* roff, int32_t ntile,
                              const double* mx, double eps, const int32_t* shell_of, int32_t nshell, int32_t* flag,
                              hipStream_t s)
{
    if (nbf <= 0 || ntile <= 0) return hipSuccess;
    if (!P || !fn || !roff || !mx || !shell_of || !flag) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ftilde_flag_kernel, dim3((unsigned)((nbf + 3) / 4), (unsigned)ntile), dim3(256), 0, s, P, nbf,
                       fn, roff, mx, eps, shell_of, nshell, flag);
    return hipGetLastError();
}

hipError_t launch_gather(const double* P, int64_t nbf, const int32_t* rows, int64_t M, const int32_t* cols, int64_t N,
                         double* out, hipStream_t s)
{
    return launch_gather_t<double>(P, nbf, rows, M, cols, N, out, s);
}

hipError_t launch_gather(const double* P, int64_t nbf, const int32_t* rows, int64_t M, const int32_t* cols, int64_t N,
                         float* out, hipStream_t s)
{
    return launch_gather_t<float>(P, nbf, rows, M, cols, N, out, s);
}

}  // namespace snk
