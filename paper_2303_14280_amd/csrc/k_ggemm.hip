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
// wave WM x WN blocks of 16 x 16; 128 x 128, 64 x 128 or 64 x 64, chosen per launch by the padded work
// of its problems), k in steps of 16 (32 for the FP32 part of a split product: the same
// matrix-core time per step as its FP64 part) staged through double-buffered LDS with the next
// step's global loads in flight during the current step's matrix-core work.  FP64 mode:
// v_mfma_f64_16x16x4f64, FP64 operands and sums.  FP32 mode: operands rounded to FP32 as they
// are staged, v_mfma_f32_16x16x4f32 with FP32 sums over the workgroup's k chunk; the host keeps
// those chunks at most kFp32MaxK long and adds chunks in FP64 (split products) or FP64
// accumulation into C.
//
// A deterministic scatter-add of the chunk products into a row-major FP64 target goes with
// it: one workgroup per target row walks the tiles in list order.
#include "snk_internal.h"

namespace snk {
namespace {

// k extent of one staged operand step (chunks of a split k are multiples of it).  The FP32 part
// of a split product stages 2 GBK: an FP32 16 x 16 x 4 product takes half the cycles of the FP64
// one, so its steps then take as long as the FP64 part's and the barrier and load latency per
// step weigh the same; the plain FP32 products keep GBK.
constexpr int GBK = 16, GPAD = 4;

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

// One operand pair of a product as the main loop reads it: A(i, k) = A[arow(i) lda + acol(k)]
// (k contiguous), B(k, j) = B[bmap(k) ldb + j] or, transposed, B[bmap(j) ldb + k].
template <typename TA, typename TB>
struct Operands {
    GP<const TA> A;
    const int32_t* arow;
    const int32_t* acol;
    int64_t lda;
    GP<const TB> B;
    const int32_t* bmap;
    int64_t ldb;
    bool avec, bvec;
};

// Row-major B is staged with one free slot after every 8 columns (column j at j + j / 8): a
// lane stages a run of 8 columns, so without the gaps the 16 lanes of a k row would start
// their runs on only two (FP64) or four (FP32) of the 32 LDS banks.  The row length then puts
// consecutive k rows 8 (FP64) or 16 (FP32) banks apart for the matrix-core operand reads.
__host__ __device__ constexpr int skew(int j) { return j + (j >> 3); }
template <typename TS>
constexpr int bcols(int bn)
{
    int c = skew(bn);
    const int target = sizeof(TS) == 8 ? 8 : 16;
    while ((c * (int)sizeof(TS) / 4) % 32 != target) ++c;
    return c;
}

// Workgroup shape: 2 x GN waves (128 GN threads), each wave WM x WN blocks of 16 x 16, so
// BM = 32 WM rows and BN = 16 WN GN columns of output.
template <int GN>
constexpr int nthreads() { return 128 * GN; }
template <int WN, int GN>
constexpr int tile_n() { return 16 * WN * GN; }

// Double-buffered LDS staging of BM x BK (A, k-major) and BK x BN (B) operand tiles.
template <typename TS, int WM, int WN, int GN, int BK = GBK>
struct Stage {
    TS A[2][BK][32 * WM + GPAD];
    TS B[2][BK][bcols<TS>(tile_n<WN, GN>())];
};

template <typename TS>
__device__ inline void mfma_step(TS a, TS b, typename GTraits<sizeof(TS) == 4 ? 1 : 0>::acc4& acc)
{
    if constexpr (sizeof(TS) == 4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    else acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// The k loop of one workgroup over [kbeg, kend) for outputs [m0, m0 + BM) x [n0, n0 + BN)
// (rows < M, columns < N): operands staged to TS (FP64 or FP32) in LDS, matrix-core products
// accumulated into acc (the wave's WM x WN blocks).  Every load address is clamped into the
// operand (k to kend - 1, columns to N - 1) and out-of-range elements are staged as zeros;
// runs that lie inside and start on 16-byte aligned rows are read as vectors.  With TAIL a
// partial last step stops after its last 4-wide k group (the staged zeros past it add nothing):
// the split product's short k ranges gain 3% from it, while the other products' long chunks
// lose up to 14% to the branch in their step loop on gfx950, so only the split product sets it.
template <typename TS, typename TA, typename TB, bool BT, int WM, int WN, int GN, int BK, bool TAIL = false>
__device__ inline void mainloop(Stage<TS, WM, WN, GN, BK>& L, const Operands<TA, TB>& op, int64_t M, int64_t N,
                                int64_t m0, int64_t n0, int64_t kbeg, int64_t kend,
                                typename GTraits<sizeof(TS) == 4 ? 1 : 0>::acc4 (&acc)[WM][WN])
{
    constexpr int NT = nthreads<GN>();
    constexpr int BM = 32 * WM, BN = tile_n<WN, GN>();
    constexpr int E = BM * BK / NT;     // A elements each thread stages per k step
    constexpr int TPR = BK / E;         // threads per k-contiguous run of BK of A
    constexpr int EB = BN * BK / NT;    // B elements each thread stages per k step
    constexpr int TPRB = BK / EB;
    static_assert(BM * BK == NT * E && BN * BK == NT * EB, "whole runs per thread");
    const int nk = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
    const GP<const int32_t> acol = glb(op.acol);
    const GP<const int32_t> bmap = glb(op.bmap);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / GN) * (BM / 2), wn = (wave % GN) * (BN / GN);
    const int li = lane & 15, lk = lane >> 4;

    // A row tid / TPR, k run (tid % TPR) * E; rows past M read row M - 1 and stage zeros
    const int ai = tid / TPR, ak = (tid % TPR) * E;
    const int64_t gma = m0 + ai;
    const bool a_ok = gma < M;
    const int64_t arow_i = a_ok ? gma : M - 1;
    const GP<const TA> arow_ptr = op.A + (int64_t)(op.arow ? glb(op.arow)[arow_i] : arow_i) * op.lda;
    // B: row-major -> k = tid / (BN / EB), columns (tid % (BN / EB)) * EB; transposed -> column
    // tid / TPRB, k run (tid % TPRB) * EB
    const int bk = BT ? (tid % TPRB) * EB : tid / (BN / EB);
    const int bj = BT ? tid / TPRB : (tid % (BN / EB)) * EB;
    TS va[E], vb[EB];

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
        } else if (op.avec && ka + E <= kend) {
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
            const bool n_ok = gn < N;
            const int64_t bn = n_ok ? gn : N - 1;
            const GP<const TB> brow = op.B + (int64_t)(bmap ? bmap[bn] : bn) * op.ldb;
            const int64_t kb = k0 + bk;
            if (op.bvec && kb + EB <= kend) {
                loadv<EB>(brow + kb, vb);
                if (!n_ok)
#pragma unroll
                    for (int u = 0; u < EB; ++u) vb[u] = (TS)0;
            } else {
#pragma unroll
                for (int u = 0; u < EB; ++u) {
                    const TS v = (TS)brow[kb + u < kend ? kb + u : kend - 1];
                    vb[u] = (n_ok && kb + u < kend) ? v : (TS)0;
                }
            }
        } else {
            const int64_t gk = k0 + bk;
            const bool k_ok = gk < kend;
            const int64_t bkk = k_ok ? gk : kend - 1;
            const GP<const TB> brow = op.B + (int64_t)(bmap ? bmap[bkk] : bkk) * op.ldb;
            const int64_t gn = n0 + bj;
            if (op.bvec && gn + EB <= N) {
                loadv<EB>(brow + gn, vb);
                if (!k_ok)
#pragma unroll
                    for (int u = 0; u < EB; ++u) vb[u] = (TS)0;
            } else {
#pragma unroll
                for (int u = 0; u < EB; ++u) {
                    const TS v = (TS)brow[gn + u < N ? gn + u : N - 1];
                    vb[u] = (k_ok && gn + u < N) ? v : (TS)0;
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < E; ++u) L.A[buf][ak + u][ai] = va[u];
        if constexpr (BT) {
#pragma unroll
            for (int u = 0; u < EB; ++u) L.B[buf][bk + u][bj] = vb[u];
        } else {
#pragma unroll
            for (int u = 0; u < EB; ++u) L.B[buf][bk][skew(bj + u)] = vb[u];
        }
    };

    if (nk > 0) {
        load(kbeg);
    } else {
#pragma unroll
        for (int u = 0; u < E; ++u) va[u] = (TS)0;
#pragma unroll
        for (int u = 0; u < EB; ++u) vb[u] = (TS)0;
    }
    store(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        // k left in this step, the same in every lane
        const int64_t kleft = kend - kbeg - (int64_t)it * BK;
        const int krem = __builtin_amdgcn_readfirstlane(kleft < BK ? (int)kleft : BK);
        if (it + 1 < nk) load(kbeg + (int64_t)(it + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            if constexpr (TAIL) {
                if (ks >= krem) break;
            }
            TS a[WM], b[WN];
#pragma unroll
            for (int bi = 0; bi < WM; ++bi) a[bi] = L.A[cur][ks + lk][wm + bi * 16 + li];
#pragma unroll
            for (int bj2 = 0; bj2 < WN; ++bj2) {
                const int j = wn + bj2 * 16 + li;
                b[bj2] = L.B[cur][ks + lk][BT ? j : skew(j)];
            }
#pragma unroll
            for (int bi = 0; bi < WM; ++bi)
#pragma unroll
                for (int bj2 = 0; bj2 < WN; ++bj2) mfma_step<TS>(a[bi], b[bj2], acc[bi][bj2]);
        }
        if (it + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }
}

// The problem and output tile of workgroup blockIdx.x.  The hardware deals consecutive
// workgroups out to the 8 XCDs in turn; workgroup w takes logical tile (w % 8) * per + w / 8,
// so each XCD works through one contiguous range of tiles (tiles that share operands share
// that XCD's L2).  Returns false for the padding workgroups of the last round.
template <int WM, int WN, int GN>
__device__ inline bool locate(const GemmProb* __restrict__ probs, int nprob, int64_t nwg, GemmProb& pr, int& z,
                              int64_t& m0, int64_t& n0)
{
    const int64_t per = gridDim.x >> 3;   // gridDim.x is a multiple of 8
    const int64_t w = blockIdx.x;
    const int64_t logical = (w & 7) * per + (w >> 3);
    if (logical >= nwg) return false;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].wg0 <= logical) lo = mid;
        else hi = mid - 1;
    }
    pr = probs[lo];
    const int local = (int)(logical - pr.wg0);   // < tm tn ksplit, far below 2^31
    const int tmn = pr.tm * pr.tn;
    z = local / tmn;
    const int rmn = local - z * tmn;
    const int tn_i = rmn / pr.tm;
    const int tm_i = rmn - tn_i * pr.tm;
    m0 = (int64_t)tm_i * 32 * WM;
    n0 = (int64_t)tn_i * tile_n<WN, GN>();
    return true;
}

// Writes the wave's blocks of acc to C (row crow(i), stride ldc), adding to C with kGemmAccumulate.
// Accumulator layouts (wave64): FP64 D[i][j] in lane j + 16 (i % 4), element i / 4; FP32
// D[i][j] in lane j + 16 (i / 4), element i % 4.
template <typename TC, int MODE, int WM, int WN, int GN, typename ACC>
__device__ inline void write_tile(const GemmProb& pr, int z, int64_t m0, int64_t n0, const ACC (&acc)[WM][WN])
{
    constexpr int BM = 32 * WM, BN = tile_n<WN, GN>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave / GN) * (BM / 2), wn = (wave % GN) * (BN / GN);
    const int li = lane & 15, lk = lane >> 4;
    const GP<TC> C = glbw(static_cast<TC*>(pr.C)) + (int64_t)z * pr.cstride;
    auto write_out = [&](auto op) {
#pragma unroll
        for (int bi = 0; bi < WM; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm + bi * 16 + (MODE == 1 ? 4 * lk + r : 4 * r + lk);
                if (gm >= pr.M) continue;
                const GP<TC> crow = C + (int64_t)(pr.crow ? glb(pr.crow)[gm] : gm) * pr.ldc;
#pragma unroll
                for (int bj2 = 0; bj2 < WN; ++bj2) {
                    const int64_t gn = n0 + wn + bj2 * 16 + li;
                    if (gn < pr.N) op(crow + gn, (TC)acc[bi][bj2][r]);
                }
            }
    };
    if (pr.vec & kGemmAccumulate) write_out([](GP<TC> q, TC v) { *q += v; });
    else write_out([](GP<TC> q, TC v) { *q = v; });
}

// WM x WN blocks of 16 x 16 per wave, 2 x GN waves: BM = 32 WM by BN = 16 WN GN outputs per
// workgroup (two workgroups of 256 threads or one of 512 per compute unit)
template <typename TA, typename TB, typename TC, int MODE, bool BT, int WM, int WN, int GN>
__global__ __launch_bounds__(nthreads<GN>(), 512 / nthreads<GN>()) void ggemm_kernel(const GemmProb* __restrict__ probs,
                                                                                      int nprob, int64_t nwg)
{
    typedef typename GTraits<MODE>::TS TS;
    typedef typename GTraits<MODE>::acc4 acc4;
    __shared__ Stage<TS, WM, WN, GN> L;
    GemmProb pr;
    int z;
    int64_t m0, n0;
    if (!locate<WM, WN, GN>(probs, nprob, nwg, pr, z, m0, n0)) return;
    const int64_t kbeg = (int64_t)z * pr.kchunk;
    const int64_t kend = kbeg + pr.kchunk < pr.K ? kbeg + pr.kchunk : pr.K;
    Operands<TA, TB> op{glb(static_cast<const TA*>(pr.A)), pr.arow, pr.acol, pr.lda,
                        glb(static_cast<const TB*>(pr.B)), pr.bmap, pr.ldb, (pr.vec & 1) != 0, (pr.vec & 2) != 0};
    acc4 acc[WM][WN];
#pragma unroll
    for (int bi = 0; bi < WM; ++bi)
#pragma unroll
        for (int bj2 = 0; bj2 < WN; ++bj2) acc[bi][bj2] = acc4{0, 0, 0, 0};
    mainloop<TS, TA, TB, BT, WM, WN, GN>(L, op, pr.M, pr.N, m0, n0, kbeg, kend, acc);
    write_tile<TC, MODE, WM, WN, GN>(pr, z, m0, n0, acc);
}

// LDS of the split product: the FP32 stage (32-deep k steps) and the FP64 stage in turn
template <int WM, int WN, int GN>
union SplitStage {
    Stage<double, WM, WN, GN> d;
    Stage<float, WM, WN, GN, 2 * GBK> f;
};

// Split product (one chunk, B row-major): C = A B over the strong k (FP64 operands, FP64 matrix
// cores) plus A2 B2 over the weak k (FP32 operands, FP32 matrix cores, K2 <= kFp32MaxK), C
// written once.  The weak sums come first: their FP32 accumulators go through LDS into the
// FP64 layout (the two accumulator layouts differ) as the starting values of the FP64 sums, so
// only one accumulator set is live at a time and the 128 x 128 tile fits in registers.
template <int WM, int WN, int GN>
__global__ __launch_bounds__(nthreads<GN>(), 512 / nthreads<GN>()) void gsplit_kernel(const GemmProb* __restrict__ probs,
                                                                                       int nprob, int64_t nwg)
{
    typedef GTraits<0>::acc4 acc64;
    typedef GTraits<1>::acc4 acc32;
    constexpr int BM = 32 * WM, BN = tile_n<WN, GN>();
    __shared__ SplitStage<WM, WN, GN> L;
    GemmProb pr;
    int z;
    int64_t m0, n0;
    if (!locate<WM, WN, GN>(probs, nprob, nwg, pr, z, m0, n0)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave / GN) * (BM / 2), wn = (wave % GN) * (BN / GN);
    const int li = lane & 15, lk = lane >> 4;
    // the transpose goes through the staging LDS in NH column parts when it cannot hold the
    // whole tile at once
    constexpr int NH = sizeof(SplitStage<WM, WN, GN>) >= sizeof(float) * BM * (BN + 1) ? 1 : 2;
    constexpr int HC = BN / NH;
    static_assert(sizeof(SplitStage<WM, WN, GN>) >= sizeof(float) * BM * (HC + 1), "LDS for the transpose");
    static_assert(BN / GN <= HC && HC % (BN / GN) == 0, "each wave's columns within one part");
    float* T = reinterpret_cast<float*>(&L);
    acc32 acw[WM][WN];
#pragma unroll
    for (int bi = 0; bi < WM; ++bi)
#pragma unroll
        for (int bj2 = 0; bj2 < WN; ++bj2) acw[bi][bj2] = acc32{0, 0, 0, 0};
    {
        Operands<float, float> op{glb(static_cast<const float*>(pr.A2)), pr.arow, nullptr, pr.lda2,
                                  glb(static_cast<const float*>(pr.B2)), nullptr, pr.ldb2, (pr.vec & 8) != 0,
                                  (pr.vec & 16) != 0};
        mainloop<float, float, float, false, WM, WN, GN, 2 * GBK, true>(L.f, op, pr.M, pr.N, m0, n0, 0, pr.K2, acw);
    }
    // FP32 blocks to LDS in (row, column) order and back in the FP64 accumulator layout (the
    // main loop ends with a barrier)
    acc64 acc[WM][WN];
    const int part = wn / HC, wc = wn - part * HC;
    for (int h = 0; h < NH; ++h) {
        if (part == h) {
#pragma unroll
            for (int bi = 0; bi < WM; ++bi)
#pragma unroll
                for (int bj2 = 0; bj2 < WN; ++bj2)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        T[(wm + bi * 16 + 4 * lk + r) * (HC + 1) + wc + bj2 * 16 + li] = acw[bi][bj2][r];
        }
        __syncthreads();
        if (part == h) {
#pragma unroll
            for (int bi = 0; bi < WM; ++bi)
#pragma unroll
                for (int bj2 = 0; bj2 < WN; ++bj2)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[bi][bj2][r] = (double)T[(wm + bi * 16 + 4 * r + lk) * (HC + 1) + wc + bj2 * 16 + li];
        }
        __syncthreads();   // the next part, then the FP64 main loop, restage the same LDS
    }
    {
        Operands<double, double> op{glb(static_cast<const double*>(pr.A)), pr.arow, pr.acol, pr.lda,
                                    glb(static_cast<const double*>(pr.B)), pr.bmap, pr.ldb, (pr.vec & 1) != 0,
                                    (pr.vec & 2) != 0};
        mainloop<double, double, double, false, WM, WN, GN, GBK, true>(L.d, op, pr.M, pr.N, m0, n0, 0, pr.K, acc);
    }
    write_tile<double, 0, WM, WN, GN>(pr, z, m0, n0, acc);
}

// One workgroup per target row r: for every tile in list order, the tile's local row of r
// (if any) summed over its chunks in chunk order and added into the row's columns.  Within a
// tile the target columns are distinct; the barrier orders tiles that share columns.  The tiles
// holding r are found 256 at a time, one lane per tile, and compacted in list order through LDS,
// so the ordered walk visits only those (a row sits in a few of a group's tiles when the basis
// is screened) instead of waiting on two dependent loads per tile.
__global__ __launch_bounds__(256) void group_reduce_kernel(const double* __restrict__ part,
                                                           const RedTile* __restrict__ tiles, int ntile,
                                                           double* __restrict__ T, int64_t ldt, int64_t nrow)
{
    __shared__ int2 hit[256];
    __shared__ int wcount[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t r = blockIdx.x; r < nrow; r += gridDim.x) {
        double* trow = T + r * ldt;
        for (int t0 = 0; t0 < ntile; t0 += 256) {
            const int t = t0 + (int)threadIdx.x;
            int i = -1;
            if (t < ntile) {
                const int32_t* rinv = tiles[t].rinv;
                i = rinv ? rinv[r] : (r < tiles[t].M ? (int)r : -1);
            }
            const uint64_t m = __ballot(i >= 0);
            if (lane == 0) wcount[wave] = __popcll(m);
            __syncthreads();
            int base = 0;
            for (int w = 0; w < wave; ++w) base += wcount[w];
            const int nh = wcount[0] + wcount[1] + wcount[2] + wcount[3];
            if (i >= 0) hit[base + __popcll(m & ((1ull << lane) - 1))] = make_int2(t, i);
            __syncthreads();
            for (int h = 0; h < nh; ++h) {
                const int2 e = hit[h];
                const RedTile tl = tiles[e.x];
                const int64_t mn = (int64_t)tl.M * tl.N;
                const double* p = part + tl.poff + (int64_t)e.y * tl.N;
                for (int n = threadIdx.x; n < tl.N; n += blockDim.x) {
                    double s = 0.0;
                    for (int zz = 0; zz < tl.ksplit; ++zz) s += p[zz * mn + n];
                    trow[tl.ccol ? tl.ccol[n] : n] += s;
                }
                __syncthreads();
            }
            __syncthreads();   // hit and wcount are rewritten by the next 256 tiles
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

// One workgroup row-chunk per tile (blockIdx.y): out[off + i ld + k] = src[row(i)][col(k)]
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void gather_tiles_kernel(const TI* __restrict__ P,
                                                           const GatherTile* __restrict__ tiles, TO* __restrict__ out)
{
    const GatherTile g = tiles[blockIdx.y];
    for (int i = blockIdx.x; i < g.M; i += gridDim.x) {
        const TI* src = P + g.src_off + (int64_t)(g.rows ? g.rows[i] : i) * g.src_ld;
        TO* dst = out + g.out_off + (int64_t)i * g.ld;
        for (int k = threadIdx.x; k < g.N; k += blockDim.x) dst[k] = (TO)src[g.cols ? g.cols[k] : k];
    }
}

// One workgroup per tile: stable partition of the tile's rows into mx >= tau, then the rest
__global__ __launch_bounds__(256) void partition_kernel(const double* __restrict__ mx, const int32_t* __restrict__ fn,
                                                        const int32_t* __restrict__ roff, double tau,
                                                        int32_t* __restrict__ perm, int32_t* __restrict__ cperm,
                                                        int32_t* __restrict__ nstrong)
{
    __shared__ int32_t scan[256];
    __shared__ int32_t base[2];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int r0 = roff[t], n = roff[t + 1] - r0;
    // pass 1: strong rows
    int cnt = 0;
    for (int r = tid; r < n; r += 256) cnt += mx[r0 + r] >= tau ? 1 : 0;
    scan[tid] = cnt;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) scan[tid] += scan[tid + st];
        __syncthreads();
    }
    const int ns = scan[0];
    __syncthreads();
    if (tid == 0) {
        base[0] = 0;
        base[1] = ns;
        // at most kFp32MaxK weak rows (FP32 sums of bounded length): the first of the others
        // join the strong ones
        nstrong[t] = ns > n - kFp32MaxK ? ns : n - kFp32MaxK;
    }
    __syncthreads();
    // pass 2: chunks of 256 rows in order, exclusive scan of the strong flags within a chunk
    for (int c0 = 0; c0 < n; c0 += 256) {
        const int r = c0 + tid;
        const int f = (r < n && mx[r0 + r] >= tau) ? 1 : 0;
        scan[tid] = f;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int incl = scan[tid];
        const int strong_before = incl - f;
        const int chunk_n = (n - c0) < 256 ? (n - c0) : 256;
        if (r < n) {
            const int pos = f ? base[0] + strong_before : base[1] + (tid - strong_before);
            perm[r0 + pos] = r;
            cperm[r0 + pos] = fn[r0 + r];
        }
        const int total_strong = scan[chunk_n - 1];
        __syncthreads();
        if (tid == 0) {
            base[0] += total_strong;
            base[1] += chunk_n - total_strong;
        }
        __syncthreads();
    }
}

constexpr int kBoundChunks = kBoundChunksPerTile;

// blockIdx.y = tile, blockIdx.x = chunk: waves take the tile's rows idx = chunk * 4 + wave
// (mod kBoundChunks * 4); out[tile * kBoundChunks + chunk] = sum over those rows of g_r p_r
__global__ __launch_bounds__(256) void lowprec_bound_kernel(const double* __restrict__ G, int64_t ld,
                                                            const double* __restrict__ P, int64_t nbf,
                                                            const BoundTile* __restrict__ tiles,
                                                            const int32_t* __restrict__ rows,
                                                            const int32_t* __restrict__ counts,
                                                            const int32_t* __restrict__ cperm,
                                                            double* __restrict__ out)
{
    __shared__ double part[4];
    const int t = blockIdx.y, chunk = blockIdx.x;
    const BoundTile bt = tiles[t];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = counts[t];
    double acc = 0.0;
    for (int idx = chunk * 4 + wave; idx < n; idx += kBoundChunks * 4) {
        const int r = rows[(int64_t)t * nbf + idx];
        const double* grow = G + (int64_t)r * ld + bt.col0;
        double g = 0.0;
        for (int i = lane; i < bt.ncols; i += 64) g += fabs(grow[i]);
        const double* prow = P + (int64_t)r * nbf;
        double p = 0.0;
        for (int k = bt.nstrong + lane; k < bt.nB; k += 64) p += fabs(prow[cperm[bt.roff + k]]);
        for (int o = 32; o > 0; o >>= 1) {
            g += __shfl_xor(g, o);
            p += __shfl_xor(p, o);
        }
        acc += g * p;
    }
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[(int64_t)t * kBoundChunks + chunk] = ((part[0] + part[1]) + part[2]) + part[3];
}

// acc[0] += sum of part[0 .. n) in a fixed order
__global__ __launch_bounds__(256) void bound_sum_kernel(const double* __restrict__ part, int64_t n,
                                                        double* __restrict__ acc)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[0] += sh[0];
}

template <int WM, int WN, int GN>
hipError_t launch_gsplit_wb(const GemmProb* probs, int nprob, int64_t nwg, hipStream_t s)
{
    const int64_t grid = ((nwg + 7) / 8) * 8;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gsplit_kernel<WM, WN, GN>), dim3((unsigned)grid), dim3(nthreads<GN>()), 0, s, probs, nprob,
                       nwg);
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC, int MODE, int WM, int WN, int GN>
hipError_t launch_ggemm_wb(const GemmProb* probs, int nprob, int64_t nwg, bool bt, hipStream_t s)
{
    const int64_t grid = ((nwg + 7) / 8) * 8;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    if (bt)
        hipLaunchKernelGGL((ggemm_kernel<TA, TB, TC, MODE, true, WM, WN, GN>), dim3((unsigned)grid),
                           dim3(nthreads<GN>()), 0, s, probs, nprob, nwg);
    else
        hipLaunchKernelGGL((ggemm_kernel<TA, TB, TC, MODE, false, WM, WN, GN>), dim3((unsigned)grid),
                           dim3(nthreads<GN>()), 0, s, probs, nprob, nwg);
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC, int MODE>
hipError_t launch_ggemm_t(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    if (nprob <= 0 || nwg <= 0) return hipSuccess;
    switch (tile) {
        case kTile64: return launch_ggemm_wb<TA, TB, TC, MODE, 2, 2, 2>(probs, nprob, nwg, bt, s);
        case kTile64x128: return launch_ggemm_wb<TA, TB, TC, MODE, 2, 4, 2>(probs, nprob, nwg, bt, s);
        case kTile128: return launch_ggemm_wb<TA, TB, TC, MODE, 4, 4, 2>(probs, nprob, nwg, bt, s);
        case kTile128x256: return launch_ggemm_wb<TA, TB, TC, MODE, 4, 4, 4>(probs, nprob, nwg, bt, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int g_force_tile = 0;

// Relative cost per padded flop of the 128 x 256 tiles (workgroups of 512 threads, one per
// compute unit): 1.01 to 1.03 of 128 x 128 on gfx950 (the split F product of the 1000-atom
// build 8.26 against 8.18 ms per launch), although they stage a third fewer operand bytes per
// flop; taken only where they save padding.
constexpr double kWideRate = 1.03;

int ggemm_tile(const GemmProb* probs, int nprob)
{
    if (g_force_tile) return g_force_tile;
    // Measured on gfx950 with the build's product shapes (FP64, two workgroups per compute
    // unit): per padded flop 64 x 128 tiles run at about 0.9 and 64 x 64 tiles at about 0.75 of
    // the rate of 128 x 128 tiles (more operand bytes per flop), so a smaller tile is taken only
    // where it saves more padding than that.
    double w64 = 0.0, w64x128 = 0.0, w128 = 0.0, w128x256 = 0.0;
    for (int i = 0; i < nprob; ++i) {
        const double k = (double)probs[i].K;
        const double m64 = (double)((probs[i].M + 63) / 64 * 64), m128 = (double)((probs[i].M + 127) / 128 * 128);
        const double n64 = (double)((probs[i].N + 63) / 64 * 64), n128 = (double)((probs[i].N + 127) / 128 * 128);
        const double n256 = (double)((probs[i].N + 255) / 256 * 256);
        w64 += m64 * n64 * k;
        w64x128 += m64 * n128 * k;
        w128 += m128 * n128 * k;
        w128x256 += m128 * n256 * k;
    }
    const double c[4] = {1.35 * w64, 1.1 * w64x128, w128, kWideRate * w128x256};
    const int tiles[4] = {kTile64, kTile64x128, kTile128, kTile128x256};
    int best = 2;
    for (int t = 0; t < 4; ++t)
        if (c[t] < c[best]) best = t;
    return tiles[best];
}

void ggemm_plan(GemmProb& p, int tile, int asize, int bsize)
{
    // 16-byte vector loads where every row start is 16-byte aligned (runs start at multiples
    // of 4 elements)
    const auto al = [](const void* q, int64_t ld, int sz) {
        return ((uintptr_t)q % 16 == 0) && ((ld * sz) % 16 == 0);
    };
    p.vec = (p.vec & kGemmAccumulate) | (al(p.A, p.lda, asize) ? 1 : 0) | (al(p.B, p.ldb, bsize) ? 2 : 0) |
            (p.A2 && al(p.A2, p.lda2, 4) ? 8 : 0) | (p.B2 && al(p.B2, p.ldb2, 4) ? 16 : 0);
    const int rows = tile_rows(tile), cols = tile_cols(tile);
    p.tm = (int32_t)((p.M + rows - 1) / rows);
    p.tn = (int32_t)((p.N + cols - 1) / cols);
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

hipError_t launch_gsplit(const GemmProb* probs, int nprob, int64_t nwg, int tile, hipStream_t s)
{
    if (nprob <= 0 || nwg <= 0) return hipSuccess;
    switch (tile) {
        case kTile64: return launch_gsplit_wb<2, 2, 2>(probs, nprob, nwg, s);
        case kTile64x128: return launch_gsplit_wb<2, 4, 2>(probs, nprob, nwg, s);
        case kTile128: return launch_gsplit_wb<4, 4, 2>(probs, nprob, nwg, s);
        case kTile128x256: return launch_gsplit_wb<4, 4, 4>(probs, nprob, nwg, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ggemm_f32_dd(const GemmProb* probs, int nprob, int64_t nwg, int tile, bool bt, hipStream_t s)
{
    return launch_ggemm_t<double, double, double, 1>(probs, nprob, nwg, tile, bt, s);
}

template <typename TI, typename TO>
hipError_t launch_gather_tiles_t(const TI* src, const GatherTile* tiles, int ntile, int32_t max_rows, TO* out,
                                 hipStream_t s)
{
    if (ntile <= 0 || max_rows <= 0) return hipSuccess;
    const unsigned gx = (unsigned)(max_rows < 1024 ? max_rows : 1024);
    hipLaunchKernelGGL((gather_tiles_kernel<TI, TO>), dim3(gx, (unsigned)ntile), dim3(256), 0, s, src, tiles, out);
    return hipGetLastError();
}

hipError_t launch_gather_tiles(const double* src, const GatherTile* tiles, int ntile, int32_t max_rows, double* out,
                               hipStream_t s)
{
    return launch_gather_tiles_t<double, double>(src, tiles, ntile, max_rows, out, s);
}

hipError_t launch_gather_tiles(const float* src, const GatherTile* tiles, int ntile, int32_t max_rows, float* out,
                               hipStream_t s)
{
    return launch_gather_tiles_t<float, float>(src, tiles, ntile, max_rows, out, s);
}

hipError_t launch_gather_tiles(const double* src, const GatherTile* tiles, int ntile, int32_t max_rows, float* out,
                               hipStream_t s)
{
    return launch_gather_tiles_t<double, float>(src, tiles, ntile, max_rows, out, s);
}

hipError_t launch_partition(const double* mx, const int32_t* fn, const int32_t* roff, int ntile, double tau,
                            int32_t* perm, int32_t* cperm, int32_t* nstrong, hipStream_t s)
{
    if (ntile <= 0) return hipSuccess;
    hipLaunchKernelGGL(partition_kernel, dim3((unsigned)ntile), dim3(256), 0, s, mx, fn, roff, tau, perm, cperm,
                       nstrong);
    return hipGetLastError();
}

hipError_t launch_lowprec_bound(const double* G, int64_t ld, const double* P, int64_t nbf, const BoundTile* tiles,
                                int ntile, const int32_t* rows, const int32_t* counts, const int32_t* cperm,
                                double* partials, double* acc, hipStream_t s)
{
    if (ntile <= 0) return hipSuccess;
    hipLaunchKernelGGL(lowprec_bound_kernel, dim3(kBoundChunks, (unsigned)ntile), dim3(256), 0, s, G, ld, P, nbf,
                       tiles, rows, counts, cperm, partials);
    hipLaunchKernelGGL(bound_sum_kernel, dim3(1), dim3(256), 0, s, partials, (int64_t)ntile * kBoundChunks, acc);
    return hipGetLastError();
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
