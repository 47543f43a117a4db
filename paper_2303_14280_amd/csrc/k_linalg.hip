// Dense linear-algebra steps of the sn-K build on gfx950 besides the grouped products
// (k_ggemm.hip):
//  - K = (Kt + Kt^T)/2 (Eq. sn_k) and E_x = -1/2 tr(P K) by a fixed two-stage tree;
//  - the bounds that restrict the rows of F per tile (row maxima of Phi, F~ flags);
//  - fill and conversion helpers, and a probe of the FP64 matrix-core accumulator layout.
#include "snk_internal.h"

#include <type_traits>

namespace snk {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

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

__global__ __launch_bounds__(256) void abs_kernel(const double* __restrict__ in, int64_t n, double* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = fabs(in[i]);
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

// Every tile of a group in one launch: workgroup (t, y) sets the rows rows[t * stride + m]
// (m = y, y + gridDim.y, .. < count[t]) of p to v over the tile's columns cols[2t] ..
// cols[2t] + cols[2t + 1] - 1.
__global__ __launch_bounds__(256) void fill_rows_tiles_kernel(double* __restrict__ p, int64_t ld,
                                                              const int32_t* __restrict__ rows, int64_t stride,
                                                              const int32_t* __restrict__ count,
                                                              const int64_t* __restrict__ cols, double v)
{
    const int t = blockIdx.x;
    const int64_t c0 = cols[2 * t], nc = cols[2 * t + 1];
    const int32_t* r = rows + (int64_t)t * stride;
    for (int64_t m = blockIdx.y; m < count[t]; m += gridDim.y) {
        double* dst = p + (int64_t)r[m] * ld + c0;
        for (int64_t c = threadIdx.x; c < nc; c += blockDim.x) dst[c] = v;
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

// One lane per (function lam, tile t): Ft = sum_k |P[lam][fn[k]]| mx[k] over the tile's
// functions (rows roff[t] .. roff[t+1]-1 of fn and mx) bounds |F_lam,i| on every point of the
// tile (Eq. fmat with |Phi_nu,i| <= mx); flag[t][shell_of[lam]] = 1 when Ft >= eps.  P is
// symmetric, so |P[lam][fn[k]]| is read as |P[fn[k]][lam]|: for each k the lanes of a wave read
// consecutive elements of one row (the tile's function index and maximum are uniform).  With a
// candidate list (cand, ncand) lane i of tile t takes lam = cand[t][i], i < ncand[t]: the
// functions not listed are those whose Ft is known to stay below eps.
__global__ __launch_bounds__(256) void ftilde_flag_kernel(const double* __restrict__ P, int64_t nbf,
                                                          const int32_t* __restrict__ fn,
                                                          const int32_t* __restrict__ roff,
                                                          const double* __restrict__ mx, double eps,
                                                          const int32_t* __restrict__ shell_of, int32_t nshell,
                                                          const int32_t* __restrict__ cand, int64_t cand_stride,
                                                          const int32_t* __restrict__ ncand,
                                                          int32_t* __restrict__ flag)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (idx >= (cand ? (int64_t)ncand[t] : nbf)) return;
    const int64_t lam = cand ? (int64_t)cand[(int64_t)t * cand_stride + idx] : idx;
    const double* col = P + lam;
    const int k0 = roff[t], k1 = roff[t + 1];
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int k = k0;
    for (; k + 3 < k1; k += 4) {
        v0 = fma(fabs(col[(int64_t)fn[k] * nbf]), mx[k], v0);
        v1 = fma(fabs(col[(int64_t)fn[k + 1] * nbf]), mx[k + 1], v1);
        v2 = fma(fabs(col[(int64_t)fn[k + 2] * nbf]), mx[k + 2], v2);
        v3 = fma(fabs(col[(int64_t)fn[k + 3] * nbf]), mx[k + 3], v3);
    }
    for (; k < k1; ++k) v0 = fma(fabs(col[(int64_t)fn[k] * nbf]), mx[k], v0);
    if ((v0 + v1) + (v2 + v3) >= eps) flag[(int64_t)t * nshell + shell_of[lam]] = 1;
}

// pmax[a][b] = max |P[lam][nu]| over the functions lam of block a and nu of block b (blocks:
// consecutive functions, blk_fn0[a] .. blk_fn0[a+1]-1); one workgroup per block a, a lane per b.
__global__ __launch_bounds__(256) void pblock_max_kernel(const double* __restrict__ P, int64_t nbf,
                                                         const int32_t* __restrict__ blk_fn0, int32_t nblk,
                                                         double* __restrict__ pmax)
{
    const int a = blockIdx.x;
    const int l0 = blk_fn0[a], l1 = blk_fn0[a + 1];
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        const int n0 = blk_fn0[b], n1 = blk_fn0[b + 1];
        double m = 0.0;
        for (int l = l0; l < l1; ++l) {
            const double* row = P + (int64_t)l * nbf;
            for (int n = n0; n < n1; ++n) m = fmax(m, fabs(row[n]));
        }
        pmax[(int64_t)a * nblk + b] = m;
    }
}

// Candidates of the F-row test of tile t (kCandSlices workgroups per tile, each taking every
// kCandSlices-th 256 blocks a): with s_b = sum of mx[k] over the tile's functions fn[k] in block
// b, every function lam of block a has
//     Ft_lam = sum_k |P[lam][fn[k]]| mx[k] <= U_a = sum_b pmax[a][b] s_b,
// so only the blocks with U_a (1 + 1e-10) >= eps (the margin covers the rounding of both sums)
// list their functions in cand[t], counted in ncand[t] (zero on entry; the list is in no
// particular order and the test of each listed function is exact).  The tile's (block, s_b)
// pairs are gathered in LDS 256 functions at a time; a tile with more than kCandBlocks of them
// lists every function.
constexpr int kCandBlocks = 1024, kCandSlices = 4;
__global__ __launch_bounds__(256) void ftilde_cand_kernel(const int32_t* __restrict__ fn,
                                                          const int32_t* __restrict__ roff,
                                                          const double* __restrict__ mx,
                                                          const int32_t* __restrict__ fn_blk,
                                                          const int32_t* __restrict__ blk_fn0, int32_t nblk,
                                                          const double* __restrict__ pmax, double eps, int64_t nbf,
                                                          int32_t* __restrict__ cand, int64_t cand_stride,
                                                          int32_t* __restrict__ ncand)
{
    __shared__ int32_t tb[kCandBlocks];
    __shared__ double ts[kCandBlocks];
    __shared__ int32_t cb[256];
    __shared__ double cm[256];
    __shared__ int32_t nb;
    const int t = blockIdx.x;
    const int k0 = roff[t], k1 = roff[t + 1];
    int32_t* out = cand + (int64_t)t * cand_stride;
    if (threadIdx.x == 0) nb = 0;
    __syncthreads();
    for (int c0 = k0; c0 < k1; c0 += 256) {
        const int k = c0 + (int)threadIdx.x;
        if (k < k1) {
            cb[threadIdx.x] = fn_blk[fn[k]];
            cm[threadIdx.x] = mx[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int n = nb;
            const int m = min(256, k1 - c0);
            for (int j = 0; j < m && n <= kCandBlocks; ++j) {
                if (n > 0 && tb[n - 1] == cb[j]) {
                    ts[n - 1] += cm[j];
                } else if (n < kCandBlocks) {
                    tb[n] = cb[j];
                    ts[n] = cm[j];
                    ++n;
                } else {
                    n = kCandBlocks + 1;   // overflow: every function is a candidate
                }
            }
            nb = n;
        }
        __syncthreads();
    }
    const int n = nb;
    if (n > kCandBlocks) {
        if (blockIdx.y == 0) {
            for (int64_t l = threadIdx.x; l < nbf; l += blockDim.x) out[l] = (int32_t)l;
            if (threadIdx.x == 0) ncand[t] = (int32_t)nbf;
        }
        return;
    }
    for (int a = blockIdx.y * blockDim.x + threadIdx.x; a < nblk; a += blockDim.x * gridDim.y) {
        const double* row = pmax + (int64_t)a * nblk;
        double u = 0.0;
#pragma unroll 8
        for (int j = 0; j < n; ++j) u = fma(row[tb[j]], ts[j], u);
        if (u * (1.0 + 1e-10) >= eps) {
            const int l0 = blk_fn0[a], l1 = blk_fn0[a + 1];
            const int pos = atomicAdd(&ncand[t], l1 - l0);
            for (int l = l0; l < l1; ++l) out[pos + (l - l0)] = l;
        }
    }
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

hipError_t launch_convert_f32(const double* in, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_abs(const double* in, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(abs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
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

hipError_t launch_fill_rows(double* p, int64_t ld, const int32_t* rows, int64_t M, int64_t ncols, double v,
                            hipStream_t s)
{
    if (M <= 0 || ncols <= 0) return hipSuccess;
    if (!p || !rows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_rows_kernel, rows_grid(M, ncols), dim3(256), 0, s, p, ld, rows, M, ncols, v);
    return hipGetLastError();
}

hipError_t launch_fill_rows_tiles(double* p, int64_t ld, const int32_t* rows, int64_t stride, const int32_t* count,
                                  const int64_t* cols, int32_t ntile, int32_t max_rows, double v, hipStream_t s)
{
    if (ntile <= 0 || max_rows <= 0) return hipSuccess;
    if (!p || !rows || !count || !cols) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_rows_tiles_kernel, dim3((unsigned)ntile, (unsigned)std::min(max_rows, 1024)), dim3(256), 0,
                       s, p, ld, rows, stride, count, cols, v);
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
                              hipStream_t s, const int32_t* cand, int64_t cand_stride, const int32_t* ncand)
{
    if (nbf <= 0 || ntile <= 0) return hipSuccess;
    if (!P || !fn || !roff || !mx || !shell_of || !flag || (cand && (!ncand || cand_stride < nbf)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(ftilde_flag_kernel, dim3((unsigned)((nbf + 255) / 256), (unsigned)ntile), dim3(256), 0, s, P, nbf,
                       fn, roff, mx, eps, shell_of, nshell, cand, cand_stride, ncand, flag);
    return hipGetLastError();
}

hipError_t launch_pblock_max(const double* P, int64_t nbf, const int32_t* blk_fn0, int32_t nblk, double* pmax,
                             hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    if (!P || !blk_fn0 || !pmax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pblock_max_kernel, dim3((unsigned)nblk), dim3(256), 0, s, P, nbf, blk_fn0, nblk, pmax);
    return hipGetLastError();
}

hipError_t launch_ftilde_cand(const int32_t* fn, const int32_t* roff, const double* mx, int32_t ntile,
                              const int32_t* fn_blk, const int32_t* blk_fn0, int32_t nblk, const double* pmax,
                              double eps, int64_t nbf, int32_t* cand, int64_t cand_stride, int32_t* ncand,
                              hipStream_t s)
{
    if (ntile <= 0) return hipSuccess;
    if (!fn || !roff || !mx || !fn_blk || !blk_fn0 || !pmax || !cand || !ncand || cand_stride < nbf)
        return hipErrorInvalidValue;
    hipError_t e = launch_fill(ncand, (int64_t)ntile, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ftilde_cand_kernel, dim3((unsigned)ntile, kCandSlices), dim3(256), 0, s, fn, roff, mx, fn_blk,
                       blk_fn0, nblk, pmax, eps, nbf, cand, cand_stride, ncand);
    return hipGetLastError();
}

}  // namespace snk
