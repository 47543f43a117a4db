// 3c-CP integral digestion for sn-K (App. A): for every shell pair (A,B) of a batch
// and every grid point r_i of it,
//   A_ab(r_i) = int phi_a phi_b / |r - r_i|                       (Eq. 3c_grid)
// is formed by the Obara-Saika vertical recursion (Eq. vrr) per primitive pair,
// contracted over primitives, taken through the horizontal recursion (Eq. hrr),
// and digested at once into G (Eq. gmat):
//   G_{a,i} += w_i sum_b A_ab(r_i) F_{b,i},   G_{b,i} += w_i sum_a A_ab(r_i) F_{a,i}  (A != B).
// The integral block is never written to memory.
//
// Work mapping (gfx950): one workgroup = one 256-point batch = four wave64 (screened
// launches: only the batches with runs, those with the most B tasks first, so that the
// heaviest workgroups do not form the launch's tail); a lane owns one grid point, so every
// G update is lane-private (no atomics and a fixed summation order).  All lanes of a wave walk the same work list, so pair
// and primitive data are wave-uniform and come through scalar loads (restrict
// kernel arguments); F/G rows move as 512-byte coalesced vectors.  A run keeps
// the F rows and G accumulators of a tile of A shells in registers while it
// sweeps the B shells, so each F_B load and G_B update serves the whole tile.
// One kernel instantiation per (l_A, l_B) class with l_A >= l_B, fully unrolled
// at compile time, per storage type of F (FP64, or FP32), and per arithmetic type: FP64,
// or FP32 for the blocks the screen marks as small enough for reduced precision (Boys
// function, recurrences and the contraction in FP32; G itself is always accumulated in
// FP64).
#include "os3c.h"

namespace snk {
namespace {

using namespace os3c;

// Grid points per lane (NP): a lane evaluates every primitive-pair record for NP points of its
// batch (workgroups of 256 / NP lanes), so that each scalar record load and loop step serves
// NP times the vector work.  Two points pay off only for the p-s class of unscreened
// launches (every batch walks the same full work list); screened launches and the other
// classes run one point per lane (measured: the extra registers cost more occupancy there).
constexpr int kPointsPerLanePs = 2;

template <int LA, int LB, int TA, int NP, typename TF, typename R>
__global__ __launch_bounds__(256) void afg_kernel(const double* __restrict__ px, const double* __restrict__ py,
                                                  const double* __restrict__ pz, const double* __restrict__ pw,
                                                  const TF* __restrict__ F, double* __restrict__ G, int64_t ld,
                                                  const typename PrimOf<R>::type* __restrict__ prims,
                                                  const int32_t* __restrict__ runs,
                                                  const int32_t* __restrict__ btasks,
                                                  const double* __restrict__ rowc,
                                                  const int32_t* __restrict__ batch_run_off, int32_t nrun,
                                                  const int32_t* __restrict__ batch_order,
                                                  const double* __restrict__ gtab)
{
    constexpr int NA = ncart(LA), NB = ncart(LB);
    constexpr int RS = 2 + TA;        // run record stride
    constexpr int BS = 2 + 2 * TA;    // B-task record stride
    constexpr int STRIDE = kBatch / NP;   // lanes per workgroup; lane t owns points t, t + STRIDE, ...
    // the Boys table columns this class reads (m + j <= l_A + l_B + terms - 1), in LDS
    constexpr int TC = LA + LB + boys_terms<R>();
    __shared__ R tab[kBoysRows * TC];
    for (int i = threadIdx.x; i < kBoysRows * TC; i += blockDim.x) tab[i] = (R)gtab[(i / TC) * kBoysCols + i % TC];
    __syncthreads();

    const int batch = batch_order ? batch_order[blockIdx.x] : (int)blockIdx.x;
    int64_t col[NP];
    R cx[NP], cy[NP], cz[NP];
    double w[NP];
    sfor<0, NP>([&](auto pc) {
        constexpr int p = CV(pc);
        col[p] = (int64_t)batch * kBatch + threadIdx.x + p * STRIDE;
        cx[p] = (R)px[col[p]];
        cy[p] = (R)py[col[p]];
        cz[p] = (R)pz[col[p]];
        w[p] = pw[col[p]];
    });

    int r0 = 0, r1 = nrun;
    if (batch_run_off) {
        r0 = batch_run_off[batch];
        r1 = batch_run_off[batch + 1];
    }
    for (int r = r0; r < r1; ++r) {
        const int32_t* run = runs + (int64_t)r * RS;
        const int b0 = run[0], b1 = run[1];
        int arow[TA];
        double RA[TA][3];   // centres of the tile's A shells (wave-uniform)
        R Fa[NP][TA][NA], Ga[NP][TA][NA];
        sfor<0, TA>([&](auto kc) {
            constexpr int k = CV(kc);
            arow[k] = run[2 + k];
            const double* ca = rowc + 3 * (int64_t)(arow[k] >= 0 ? arow[k] : 0);
            RA[k][0] = ca[0];
            RA[k][1] = ca[1];
            RA[k][2] = ca[2];
            sfor<0, NP>([&](auto pc) {
                constexpr int p = CV(pc);
                sfor<0, NA>([&](auto ic) {
                    constexpr int i = CV(ic);
                    Fa[p][k][i] = arow[k] >= 0 ? (R)(cnorm(LA, i) * (double)F[(int64_t)(arow[k] + i) * ld + col[p]])
                                               : (R)0;
                    Ga[p][k][i] = (R)0;
                });
            });
        });
        // the F_B / G_B rows of the next B task are fetched one task ahead
        int nrow = 0;
        double Fn[NP][NB], Gn[NP][NB];
        auto fetch = [&](int bt) {
            nrow = btasks[(int64_t)bt * BS];
            sfor<0, NP>([&](auto pc) {
                constexpr int p = CV(pc);
                sfor<0, NB>([&](auto jc) {
                    const int64_t o = (int64_t)(nrow + CV(jc)) * ld + col[p];
                    Fn[p][CV(jc)] = (double)F[o];
                    Gn[p][CV(jc)] = G[o];
                });
            });
        };
        if (b0 < b1) fetch(b0);
        for (int bt = b0; bt < b1; ++bt) {
            const int32_t* cur = btasks + (int64_t)bt * BS;
            const int brow = nrow;
            R Fb[NP][NB], Gb[NP][NB];
            double Gold[NP][NB];
            sfor<0, NP>([&](auto pc) {
                constexpr int p = CV(pc);
                sfor<0, NB>([&](auto jc) {
                    constexpr int j = CV(jc);
                    Fb[p][j] = (R)(cnorm(LB, j) * Fn[p][j]);
                    Gold[p][j] = Gn[p][j];
                    Gb[p][j] = (R)0;
                });
            });
            if (bt + 1 < b1) fetch(bt + 1);
            const int mask = cur[1];
            const double* cb = rowc + 3 * (int64_t)brow;
            const double RB[3] = {cb[0], cb[1], cb[2]};
            bool transposed = false;
            sfor<0, TA>([&](auto kc) {
                constexpr int k = CV(kc);
                if (mask & (1 << k)) {
                    const R AB[3] = {(R)(RA[k][0] - RB[0]), (R)(RA[k][1] - RB[1]), (R)(RA[k][2] - RB[2])};
                    R Ab[NP][NA][NB];
                    pair_block_n<LA, LB, R, NP, TC>(prims + cur[2 + 2 * k], cur[3 + 2 * k], AB, cx, cy, cz, tab, Ab);
                    const bool offdiag = arow[k] != brow;   // A != B: the transposed block feeds G_B
                    transposed |= offdiag;
                    sfor<0, NP>([&](auto pc) {
                        constexpr int p = CV(pc);
                        sfor<0, NA>([&](auto ic) {
                            constexpr int i = CV(ic);
                            R acc = Ga[p][k][i];
                            sfor<0, NB>([&](auto jc) { acc = fma(Ab[p][i][CV(jc)], Fb[p][CV(jc)], acc); });
                            Ga[p][k][i] = acc;
                        });
                        if (offdiag) {
                            sfor<0, NB>([&](auto jc) {
                                constexpr int j = CV(jc);
                                R acc = Gb[p][j];
                                sfor<0, NA>([&](auto ic) { acc = fma(Ab[p][CV(ic)][j], Fa[p][k][CV(ic)], acc); });
                                Gb[p][j] = acc;
                            });
                        }
                    });
                }
            });
            if (transposed) {
                sfor<0, NP>([&](auto pc) {
                    constexpr int p = CV(pc);
                    sfor<0, NB>([&](auto jc) {
                        constexpr int j = CV(jc);
                        G[(int64_t)(brow + j) * ld + col[p]] = fma(w[p] * cnorm(LB, j), (double)Gb[p][j], Gold[p][j]);
                    });
                });
            }
        }
        sfor<0, TA>([&](auto kc) {
            constexpr int k = CV(kc);
            if (arow[k] >= 0) {
                sfor<0, NP>([&](auto pc) {
                    constexpr int p = CV(pc);
                    sfor<0, NA>([&](auto ic) {
                        constexpr int i = CV(ic);
                        G[(int64_t)(arow[k] + i) * ld + col[p]] += (w[p] * cnorm(LA, i)) * (double)Ga[p][k][i];
                    });
                });
            }
        });
    }
}

template <int MMAX>
__global__ __launch_bounds__(256) void boys_eval_kernel(const double* __restrict__ T, int64_t n, double* __restrict__ F,
                                                        const double* __restrict__ gtab)
{
    __shared__ double tab[kBoysRows * kBoysCols];
    for (int i = threadIdx.x; i < kBoysRows * kBoysCols; i += blockDim.x) tab[i] = gtab[i];
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f[MMAX + 1];
    boys<MMAX, double>(T[k], tab, f);
    sfor<0, MMAX + 1>([&](auto mc) { F[k * (MMAX + 1) + CV(mc)] = f[CV(mc)]; });
}

}  // namespace

hipError_t launch_afg(int la, int lb, const AfgArgs& a, hipStream_t s)
{
    if (a.nbatch <= 0) return hipSuccess;
    dim3 grid(a.nbatch);
    const bool two = la == 1 && lb == 0 && a.batch_run_off == nullptr;
#define SNK_AFG_NP(LA, LB, TA, NP, TF, R, FP, PR)                                                                  \
    hipLaunchKernelGGL((afg_kernel<LA, LB, TA, NP, TF, R>), grid, dim3(kBatch / NP), 0, s, a.px, a.py, a.pz, a.pw, \
                       FP, a.G, a.ld, PR, a.runs, a.btasks, a.rowc, a.batch_run_off, a.nrun, a.batch_order,    \
                       a.boys_tab)
#define SNK_AFG_T(LA, LB, TA, TF, R, FP, PR)                                                                       \
    do {                                                                                                          \
        if (two)                                                                                                  \
            SNK_AFG_NP(LA, LB, TA, (LA == 1 && LB == 0 ? kPointsPerLanePs : 1), TF, R, FP, PR);                   \
        else                                                                                                      \
            SNK_AFG_NP(LA, LB, TA, 1, TF, R, FP, PR);                                                             \
    } while (0)
#define SNK_AFG(LA, LB, TA, TA32)                                                                       \
    if (a.lowp) {                                                                                       \
        if (a.F32)                                                                                      \
            SNK_AFG_T(LA, LB, TA32, float, float, a.F32, a.prims32);                                    \
        else                                                                                            \
            SNK_AFG_T(LA, LB, TA32, double, float, a.F, a.prims32);                                     \
    } else {                                                                                            \
        if (a.F32)                                                                                      \
            SNK_AFG_T(LA, LB, TA, float, double, a.F32, a.prims);                                       \
        else                                                                                            \
            SNK_AFG_T(LA, LB, TA, double, double, a.F, a.prims);                                        \
    }
    switch (la * 3 + lb) {
        case 0: SNK_AFG(0, 0, kTileA[0], kTileA32[0]); break;
        case 3: SNK_AFG(1, 0, kTileA[1], kTileA32[1]); break;
        case 4: SNK_AFG(1, 1, kTileA[2], kTileA32[2]); break;
        case 6: SNK_AFG(2, 0, kTileA[3], kTileA32[3]); break;
        case 7: SNK_AFG(2, 1, kTileA[4], kTileA32[4]); break;
        case 8: SNK_AFG(2, 2, kTileA[5], kTileA32[5]); break;
        default: return hipErrorInvalidValue;
    }
#undef SNK_AFG
#undef SNK_AFG_T
#undef SNK_AFG_NP
    return hipGetLastError();
}

hipError_t launch_boys_eval(const double* T, int64_t n, int mmax, double* F, const double* tab, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (mmax) {
        case 0: hipLaunchKernelGGL((boys_eval_kernel<0>), grid, block, 0, s, T, n, F, tab); break;
        case 1: hipLaunchKernelGGL((boys_eval_kernel<1>), grid, block, 0, s, T, n, F, tab); break;
        case 2: hipLaunchKernelGGL((boys_eval_kernel<2>), grid, block, 0, s, T, n, F, tab); break;
        case 3: hipLaunchKernelGGL((boys_eval_kernel<3>), grid, block, 0, s, T, n, F, tab); break;
        case 4: hipLaunchKernelGGL((boys_eval_kernel<4>), grid, block, 0, s, T, n, F, tab); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace snk
