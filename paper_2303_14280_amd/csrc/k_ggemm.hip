// Grouped GEMM on the gfx950 matrix cores: one launch evaluates a list of independent
// products of different shapes (every tile of a batch group), the device-saturating batched
// products of Sec. II.F.  Used for F = P Phi (Eq. fmat) with the rows L_t and columns B_t of
// P gathered on the fly and F scattered into the group's rows, for the split products
// G Phi^T (Eq. usym_k, Eq. vxc_num), and by the XC build.
//
// Each problem computes, for i < M, j < N and the k range of its chunk z,
//     C[z][crow(i)][j] = sum_k A(arow(i), acol(k)) B(k, j)
// with A row-major (k contiguous), B either row-major (B(k, j) = B[k ldb + j]) or read
// transposed (B(k, j) = B[j ldb + k]).  Chunks partition k; each writes its own slice of C.
//
// Tiles: BM x BN outputs per workgroup of 256 threads (four wave64 in a 2 x 2 layout, each
// wave WB x WB blocks of 16 x 16; 128 x 128 or 64 x 64, chosen per launch by the padded work
// of its problems), k in steps of 16 staged through double-buffered LDS with the next step's
// global loads in flight during the current step's matrix-core work.  FP64 mode:
// v_mfma_f64_16x16x4f64, FP64 operands and sums.  FP32 mode: operands rounded to FP32 as they
// are staged, v_mfma_f32_16x16x4f32 with FP32 sums over at most kFlushK consecutive k, added
// into FP64 sums.
//
// A deterministic scatter-add of the chunk products into a row-major FP64 target goes with
// it: one workgroup per target row walks the tiles in list order.
#include "snk_internal.h"

namespace snk {
namespace {

constexpr int GBK = 16, GPAD = 4;
constexpr int kFlushK = 1024;

template <int MODE>
struct GTraits;
template <>
struct GTraits<0> {
    typedef double TS;
    typedef double acc4 __attribute__((ext_vector_type(4)));
};
template <>
struct GTraits<1> {
    typedef float TS;
    typedef float acc4 __attribute__((ext_vector_type(4)));
};

// Pointers into global memory: the operands' addresses come out of the problem records, so
// the compiler cannot infer their address space; global loads and stores are made explicit.
template <typename T>
using GP = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline GP<const T> glb(const T* p)
{
    return (GP<const T>)p;
}
template <typename T>
__device__ inline GP<T> glbw(T* p)
{
    return (GP<T>)p;
}

// E consecutive elements from a 16-byte aligned address, as 16-byte vector loads
template <int E, typename T, typename TS>
__device__ inline void loadv(GP<const T> p, TS* out)
{
    constexpr int W = 16 / sizeof(T);
    static_assert(E % W == 0, "whole vectors only");
    typedef T v16 __attribute__((ext_vector_type(W)));
    const GP<const v16> q = (GP<const v16>)p;
#pragma unroll
    for (int h = 0; h < E / W; ++h) {
        const v16 x = q[h];
#pragma unroll
        for (int u = 0; u < W; ++u) out[h * W + u] = (TS)x[u];
    }
}

// WB x WB blocks of 16 x 16 per wave, 2 x 2 waves: BM = BN = 32 WB outputs per workgroup
template <typename TA, typename TB, typename TC, int MODE, bool BT, int WB>
__global__ __launch_bounds__(256) void ggemm_kernel(const GemmProb* __restrict__ probs, int nprob, int64_t nwg)
{
    typedef typename GTraits<MODE>::TS TS;
    typedef typename GTraits<MODE>::acc4 acc4;
    constexpr int BM = 32 * WB, BN = 32 * WB;
    constexpr int E = BM * GBK / 256;   // operand elements each thread stages per k step
    constexpr int TPR = GBK / E;        // threads per k-contiguous run of 16
    __shared__ TS As[2][GBK][BM + GPAD];
    __shared__ TS Bs[2][GBK][BN + GPAD];

    // The hardware deals consecutive workgroups out to the 8 XCDs in turn; workgroup w takes
    // logical tile (w % 8) * per + w / 8, so each XCD works through one contiguous range of
    // tiles (tiles that share operands share that XCD's L2).
    const int64_t per = gridDim.x >> 3;   // gridDim.x is a multiple of 8
    const int64_t w = blockIdx.x;
    const int64_t logical = (w & 7) * per + (w >> 3);
    if (logical >= nwg) return;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].wg0 <= logical) lo = mid;
        else hi = mid - 1;
    }
    const GemmProb pr = probs[lo];
    const int local = (int)(logical - pr.wg0);   // < tm tn ksplit, far below 2^31
    const int tmn = pr.tm * pr.tn;
    const int z = local / tmn;
    const int rmn = local - z * tmn;
    const int tn_i = rmn / pr.tm;
    const int tm_i = rmn - tn_i * pr.tm;
    const int64_t m0 = (int64_t)tm_i * BM, n0 = (int64_t)tn_i * BN;
    const int64_t kbeg = (int64_t)z * pr.kchunk;
    const int64_t kend = kbeg + pr.kchunk < pr.K ? kbeg + pr.kchunk : pr.K;
    const int nk = kend > kbeg ? (int)((kend - kbeg + GBK - 1) / GBK) : 0;

    const GP<const TA> A = glb(static_cast<const TA*>(pr.A));
    const GP<const TB> B = glb(static_cast<const TB*>(pr.B));
    const GP<const int32_t> acol = glb(pr.acol);
    const bool avec = (pr.vec & 1) != 0, bvec = (pr.vec & 2) != 0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    const int li = lane & 15, lk = lane >> 4;

    // global -> register staging: A row tid / TPR, k run (tid % TPR) * E; rows past M read
    // row M - 1 and stage zeros
    const int ai = tid / TPR, ak = (tid % TPR) * E;
    const int64_t gma = m0 + ai;
    const bool a_ok = gma < pr.M;
    const int64_t arow_i = a_ok ? gma : pr.M - 1;
    const GP<const TA> arow_ptr = A + (int64_t)(pr.arow ? glb(pr.arow)[arow_i] : arow_i) * pr.lda;
    // B: row-major -> k = tid / (BN / E), columns (tid % (BN / E)) * E; transposed -> column
    // tid / TPR, k run (tid % TPR) * E
    const int bk = BT ? (tid % TPR) * E : tid / (BN / E);
    const int bj = BT ? tid / TPR : (tid % (BN / E)) * E;
    TS va[E], vb[E];

    // Every load address is clamped into the operand (k to kend - 1, columns to N - 1) and
    // out-of-range elements are staged as zeros; runs that lie inside and start on 16-byte
    // aligned rows are read as vectors.
    auto load = [&](int64_t k0) {
        const int64_t ka = k0 + ak;
        if (acol) {
            int32_t col[E];
#pragma unroll
            for (int u = 0; u < E; ++u) col[u] = acol[ka + u < kend ? ka + u : kend - 1];
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const TS v = (TS)arow_ptr[col[u]];
                va[u] = (a_ok && ka + u < kend) ? v : (TS)0;
            }
        } else if (avec && ka + E <= kend) {
            loadv<E>(arow_ptr + ka, va);
            if (!a_ok)
#pragma unroll
                for (int u = 0; u < E; ++u) va[u] = (TS)0;
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const TS v = (TS)arow_ptr[ka + u < kend ? ka + u : kend - 1];
                va[u] = (a_ok && ka + u < kend) ? v : (TS)0;
            }
        }
        if constexpr (BT) {
            const int64_t gn = n0 + bj;
            const bool n_ok = gn < pr.N;
            const GP<const TB> brow = B + (n_ok ? gn : pr.N - 1) * pr.ldb;
            const int64_t kb = k0 + bk;
            if (bvec && kb + E <= kend) {
                loadv<E>(brow + kb, vb);
                if (!n_ok)
#pragma unroll
                    for (int u = 0; u < E; ++u) vb[u] = (TS)0;
            } else {
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const TS v = (TS)brow[kb + u < kend ? kb + u : kend - 1];
                    vb[u] = (n_ok && kb + u < kend) ? v : (TS)0;
                }
            }
        } else {
            const int64_t gk = k0 + bk;
            const bool k_ok = gk < kend;
            const GP<const TB> brow = B + (k_ok ? gk : kend - 1) * pr.ldb;
            const int64_t gn = n0 + bj;
            if (bvec && gn + E <= pr.N) {
                loadv<E>(brow + gn, vb);
                if (!k_ok)
#pragma unroll
                    for (int u = 0; u < E; ++u) vb[u] = (TS)0;
            } else {
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const TS v = (TS)brow[gn + u < pr.N ? gn + u : pr.N - 1];
                    vb[u] = (k_ok && gn + u < pr.N) ? v : (TS)0;
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < E; ++u) As[buf][ak + u][ai] = va[u];
        if constexpr (BT) {
#pragma unroll
            for (int u = 0; u < E; ++u) Bs[buf][bk + u][bj] = vb[u];
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u) Bs[buf][bk][bj + u] = vb[u];
        }
    };

    acc4 acc[WB][WB];
#pragma unroll
    for (int bi = 0; bi < WB; ++bi)
#pragma unroll
        for (int bj2 = 0; bj2 < WB; ++bj2) acc[bi][bj2] = acc4{0, 0, 0, 0};
    double dacc[WB][WB][4];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int bi = 0; bi < WB; ++bi)
#pragma unroll
            for (int bj2 = 0; bj2 < WB; ++bj2)
#pragma unroll
                for (int r = 0; r < 4; ++r) dacc[bi][bj2][r] = 0.0;
    }
    auto flush = [&]() {
        if constexpr (MODE == 1) {
#pragma unroll
            for (int bi = 0; bi < WB; ++bi)
#pragma unroll
                for (int bj2 = 0; bj2 < WB; ++bj2) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) dacc[bi][bj2][r] += (double)acc[bi][bj2][r];
                    acc[bi][bj2] = acc4{0, 0, 0, 0};
                }
        }
    };

    if (nk > 0) load(kbeg);
    else
#pragma unroll
        for (int u = 0; u < E; ++u) va[u] = vb[u] = (TS)0;
    store(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        if (it + 1 < nk) load(kbeg + (int64_t)(it + 1) * GBK);
        if (MODE == 1 && it > 0 && (it % (kFlushK / GBK)) == 0) flush();
#pragma unroll
        for (int ks = 0; ks < GBK; ks += 4) {
            TS a[WB], b[WB];
#pragma unroll
            for (int bi = 0; bi < WB; ++bi) a[bi] = As[cur][ks + lk][wm + bi * 16 + li];
#pragma unroll
            for (int bj2 = 0; bj2 < WB; ++bj2) b[bj2] = Bs[cur][ks + lk][wn + bj2 * 16 + li];
#pragma unroll
            for (int bi = 0; bi < WB; ++bi)
#pragma unroll
                for (int bj2 = 0; bj2 < WB; ++bj2) {
                    if constexpr (MODE == 1)
                        acc[bi][bj2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj2], acc[bi][bj2], 0, 0, 0);
                    else
                        acc[bi][bj2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj2], acc[bi][bj2], 0, 0, 0);
                }
        }
        if (it + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }
    flush();

    // accumulator layouts (wave64): FP64 D[i][j] in lane j + 16 (i % 4), element i / 4;
    // FP32 D[i][j] in lane j + 16 (i / 4), element i % 4
    const GP<TC> C = glbw(static_cast<TC*>(pr.C)) + (int64_t)z * pr.cstride;
#pragma unroll
    for (int bi = 0; bi < WB; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gm = m0 + wm + bi * 16 + (MODE == 1 ? 4 * lk + r : 4 * r + lk);
            if (gm >= pr.M) continue;
            const GP<TC> crow = C + (int64_t)(pr.crow ? glb(pr.crow)[gm] : gm) * pr.ldc;
#pragma unroll
            for (int bj2 = 0; bj2 < WB; ++bj2) {
                const int64_t gn = n0 + wn + bj2 * 16 + li;
                if (gn >= pr.N) continue;
                if constexpr (MODE == 1) crow[gn] = (TC)dacc[bi][bj2][r];
                else crow[gn] = (TC)acc[bi][bj2][r];
            }
        }
}

// One workgroup per target row r: for every tile in list order, the tile's local row of r
// (if any) summed over its chunks in chunk order and added into the row's columns.  Within a
// tile the target columns are distinct; the barrier orders tiles that share columns.
__global__ __launch_bounds__(256) void group_reduce_kernel(const double* __restrict__ part,
                                                           const RedTile* __restrict__ tiles, int ntile,
                                                           double* __restrict__ T, int64_t ldt, int64_t nrow)
{
    for (int64_t r = blockIdx.x; r < nrow; r += gridDim.x) {
        double* trow = T + r * ldt;
        for (int t = 0; t < ntile; ++t) {
            const RedTile tl = tiles[t];
            const int i = tl.rinv ? tl.rinv[r] : (r < tl.M ? (int)r : -1);
            if (i < 0) continue;   // uniform over the workgroup
            const int64_t mn = (int64_t)tl.M * tl.N;
            const double* p = part + tl.poff + (int64_t)i * tl.N;
            for (int n = threadIdx.x; n < tl.N; n += blockDim.x) {
                double s = 0.0;
                for (int zz = 0; zz < tl.ksplit; ++zz) s += p[zz * mn + n];
                trow[tl.ccol ? tl.ccol[n] : n] += s;
            }
            __syncthreads();
        }
    }
}

// rinv[t][r] = i for the i-th entry r of tile t's row list (entries: lists[roff[t] ..
// roff[t+1]) when roff is given, else lists[t * stride .. t * stride + counts[t]))
__global__ __launch_bounds__(256) void rinv_kernel(const int32_t* __restrict__ lists, int64_t stride,
                                                   const int32_t* __restrict__ roff,
                                                   const int32_t* __restrict__ counts, int64_t nbf,
                                                   int32_t* __restrict__ rinv)
{
    const int t = blockIdx.y;
    const int64_t b = roff ? roff[t] : (int64_t)t * stride;
    const int n = roff ? roff[t + 1] - roff[t] : counts[t];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rinv[(int64_t)t * nbf + lists[b + i]] = i;
}

template <typename TA, typename TB, typename TC, int MODE, int WB>
hipError_t launch_ggemm_wb(const GemmProb* probs, int nprob, int64_t nwg, bool bt, hipStream_t s)
{
    const int64_t grid = ((nwg + 7) / 8) * 8;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    if (bt)
        hipLaunchKernelGGL((ggemm_kernel<TA, TB, TC, MODE, true, WB>), dim3((unsigned)grid), dim3(256), 0, s, probs,
                           nprob, nwg);
    else
        hipLaunchKernelGGL((ggemm_kernel<TA, TB, TC, MODE, false, WB>), dim3((unsigned)grid), dim3(256), 0, s, probs,
                           nprob, nwg);
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC, int MODE>
hipError_t launch_ggemm_t(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    if (nprob <= 0 || nwg <= 0) return hipSuccess;
    if (tile != 64 && tile != 128) return hipErrorInvalidValue;
    return tile == 64 ? launch_ggemm_wb<TA, TB, TC, MODE, 2>(probs, nprob, nwg, bt, s)
                      : launch_ggemm_wb<TA, TB, TC, MODE, 4>(probs, nprob, nwg, bt, s);
}

}  // namespace

int ggemm_tile(const GemmProb* probs, int nprob)
{
    // Measured on gfx950: with k per workgroup of a few hundred the 64 x 64 tiles are faster
    // (four times the workgroups in flight hide the short loops' prologue and stores); with long
    // k the 128 x 128 tiles run about 1.9 times as many matrix-core flops per second, so the
    // small tiles pay only where they save that much padding.
    double w64 = 0.0, w128 = 0.0, kw = 0.0, ksum = 0.0;
    for (int i = 0; i < nprob; ++i) {
        const double k = (double)probs[i].K;
        const double ks = (double)(probs[i].ksplit > 0 ? probs[i].ksplit : 1);
        w64 += (double)((probs[i].M + 63) / 64 * 64) * (double)((probs[i].N + 63) / 64 * 64) * k;
        w128 += (double)((probs[i].M + 127) / 128 * 128) * (double)((probs[i].N + 127) / 128 * 128) * k;
        kw += k / ks * k;
        ksum += k;
    }
    const double kchunk = ksum > 0.0 ? kw / ksum : 0.0;   // work-weighted k per workgroup
    if (kchunk <= 512.0) return 64;
    return 1.9 * w64 < w128 ? 64 : 128;
}

void ggemm_plan(GemmProb& p, int tile, int asize, int bsize)
{
    // 16-byte vector loads where every row start is 16-byte aligned (runs start at multiples
    // of 4 elements)
    const auto al = [](const void* q, int64_t ld, int sz) {
        return ((uintptr_t)q % 16 == 0) && ((ld * sz) % 16 == 0);
    };
    p.vec = (al(p.A, p.lda, asize) ? 1 : 0) | (al(p.B, p.ldb, bsize) ? 2 : 0);
    p.tm = (int32_t)((p.M + tile - 1) / tile);
    p.tn = (int32_t)((p.N + tile - 1) / tile);
    if (p.ksplit < 1) p.ksplit = 1;
    int64_t kc = (p.K + p.ksplit - 1) / p.ksplit;
    kc = ((kc + GBK - 1) / GBK) * GBK;
    p.kchunk = (int32_t)(kc > 0 ? kc : GBK);
}

int64_t ggemm_workgroups(const GemmProb& p) { return (int64_t)p.tm * p.tn * p.ksplit; }

hipError_t launch_ggemm_f64(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    return launch_ggemm_t<double, double, double, 0>(probs, nprob, nwg, tile, bt, s);
}

hipError_t launch_ggemm_f32(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    return launch_ggemm_t<float, float, float, 1>(probs, nprob, nwg, tile, bt, s);
}

hipError_t launch_ggemm_f32_dA(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    return launch_ggemm_t<double, float, double, 1>(probs, nprob, nwg, tile, bt, s);
}

hipError_t launch_group_reduce(const double* part, const RedTile* tiles, int ntile, double* T, int64_t ldt,
                               int64_t nrow, hipStream_t s)
{
    if (ntile <= 0 || nrow <= 0) return hipSuccess;
    const int64_t grid = nrow < 65536 ? nrow : 65536;
    hipLaunchKernelGGL(group_reduce_kernel, dim3((unsigned)grid), dim3(256), 0, s, part, tiles, ntile, T, ldt, nrow);
    return hipGetLastError();
}

hipError_t launch_rinv(const int32_t* lists, int64_t stride, const int32_t* roff, const int32_t* counts, int ntile,
                       int64_t nbf, int64_t max_count, int32_t* rinv, hipStream_t s)
{
    if (ntile <= 0 || nbf <= 0) return hipSuccess;
    hipError_t e = launch_fill(rinv, (int64_t)ntile * nbf, -1, s);
    if (e != hipSuccess) return e;
    const int64_t gx = max_count <= 0 ? 1 : (max_count + 255) / 256 < 64 ? (max_count + 255) / 256 : 64;
    hipLaunchKernelGGL(rinv_kernel, dim3((unsigned)gx, (unsigned)ntile), dim3(256), 0, s, lists, stride, roff, counts,
                       nbf, rinv);
    return hipGetLastError();
}

}  // namespace snk
