// 3c-CP integral digestion for sn-K (App. A): for every shell pair (A,B) of a batch
// and every grid point r_i of it,
//   A_ab(r_i) = int phi_a phi_b / |r - r_i|                       (Eq. 3c_grid)
// is formed by the Obara-Saika vertical recursion (Eq. vrr) per primitive pair,
// contracted over primitives, taken through the horizontal recursion (Eq. hrr),
// and digested at once into G (Eq. gmat):
//   G_{a,i} += w_i sum_b A_ab(r_i) F_{b,i},   G_{b,i} += w_i sum_a A_ab(r_i) F_{a,i}  (A != B).
// The integral block is never written to memory.
//
// Work mapping (gfx950): one workgroup = one 256-point batch = four wave64; a
// lane owns one grid point, so every G update is lane-private (no atomics and a
// fixed summation order).  All lanes of a wave walk the same work list, so pair
// and primitive data are wave-uniform and come through scalar loads (restrict
// kernel arguments); F/G rows move as 512-byte coalesced vectors.  A run keeps
// the F rows and G accumulators of a tile of A shells in registers while it
// sweeps the B shells, so each F_B load and G_B update serves the whole tile.
// One kernel instantiation per (l_A, l_B) class with l_A >= l_B, fully unrolled
// at compile time.
#include "snk_internal.h"

#include <type_traits>

namespace snk {
namespace {

constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian exponent of direction q (0=x,1=y,2=z) of component c of level l,
// lexicographic order (x,y,z; xx,xy,xz,yy,yz,zz; ...).
constexpr int comp(int l, int c, int q)
{
    int k = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == c) return q == 0 ? x : (q == 1 ? y : l - x - y);
            ++k;
        }
    return -1;
}
constexpr int cidx(int l, int x, int z) { return ((l - x) * (l - x + 1)) / 2 + z; }
// index at level l-1 of component c (level l) lowered in direction q
constexpr int lower(int l, int c, int q)
{
    return cidx(l - 1, comp(l, c, 0) - (q == 0), comp(l, c, 2) - (q == 2));
}
// index at level l+1 of component c (level l) raised in direction q
constexpr int raise(int l, int c, int q)
{
    return cidx(l + 1, comp(l, c, 0) + (q == 0), comp(l, c, 2) + (q == 2));
}
// recursion direction: first non-zero Cartesian exponent
constexpr int dir_of(int l, int c) { return comp(l, c, 0) > 0 ? 0 : (comp(l, c, 1) > 0 ? 1 : 2); }
// factor scaling component c of a shell of angular momentum l to unit norm (l <= 2)
constexpr double cnorm(int l, int c)
{
    return (l == 2 && (c == 1 || c == 2 || c == 4)) ? 1.7320508075688772 : 1.0;
}

template <int B, int E, typename Fn>
__device__ __forceinline__ void sfor(Fn&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}
#define CV(x) decltype(x)::value

// F_m(T), m = 0..L (Eq. boys).  T < kBoysTmax: Taylor series about the nearest
// table node, F_m(T) = sum_j F_{m+j}(T_k) (T_k - T)^j / j!  (dF_m/dT = -F_{m+1});
// above: F_0 = sqrt(pi/T)/2, F_m = F_{m-1} (2m-1)/(2T).
template <int L>
__device__ __forceinline__ void boys(double T, const double* __restrict__ tab, double (&F)[L + 1])
{
    if (T < kBoysTmax) {
        const int k = (int)(T * (1.0 / kBoysStep) + 0.5);
        const double d = k * kBoysStep - T;
        const double* row = tab + k * kBoysCols;
        double pw[kBoysTerms];
        pw[0] = 1.0;
        sfor<1, kBoysTerms>([&](auto jc) {
            constexpr int j = CV(jc);
            pw[j] = pw[j - 1] * (d * (1.0 / j));
        });
        sfor<0, L + 1>([&](auto mc) {
            constexpr int m = CV(mc);
            double s = row[m + kBoysTerms - 1] * pw[kBoysTerms - 1];
            sfor<0, kBoysTerms - 1>([&](auto jc) {
                constexpr int j = kBoysTerms - 2 - CV(jc);
                s = fma(row[m + j], pw[j], s);
            });
            F[m] = s;
        });
    } else {
        const double r = rsqrt(T);
        const double h = 0.5 * r * r;
        F[0] = 0.88622692545275801365 * r;
        sfor<1, L + 1>([&](auto mc) {
            constexpr int m = CV(mc);
            F[m] = F[m - 1] * ((2 * m - 1) * h);
        });
    }
}

// Eq. vrr: Theta^n_{a+1q} = PA_q Theta^n_a - PC_q Theta^{n+1}_a + a_q/(2 zeta_p) (Theta^n_{a-1q} - Theta^{n+1}_{a-1q})
template <int L>
__device__ __forceinline__ void vrr(double (&th)[L + 1][L + 1][16], const double (&PA)[3], const double (&PC)[3],
                                    double oo2zp)
{
    sfor<1, L + 1>([&](auto lc) {
        constexpr int l = CV(lc);
        sfor<0, ncart(l)>([&](auto cc) {
            constexpr int c = CV(cc);
            constexpr int q = dir_of(l, c);
            constexpr int c1 = lower(l, c, q);
            constexpr int am = comp(l, c, q) - 1;
            constexpr int c2 = am > 0 ? lower(l - 1, c1, q) : 0;
            sfor<0, L - l + 1>([&](auto nc) {
                constexpr int n = CV(nc);
                double v = PA[q] * th[n][l - 1][c1] - PC[q] * th[n + 1][l - 1][c1];
                if constexpr (am > 0) v += (am * oo2zp) * (th[n][l - 2][c2] - th[n + 1][l - 2][c2]);
                th[n][l][c] = v;
            });
        });
    });
}

// Eq. hrr: Xi_{a(b+1q)} = Xi_{(a+1q)b} + AB_q Xi_{ab}, from Xi_{a0} = contracted Theta^0_a
template <int LA, int LB>
__device__ __forceinline__ void hrr(const double (&acc)[LA + LB + 1][16], const double (&AB)[3],
                                    double (&out)[ncart(LA)][ncart(LB)])
{
    double xi[LB + 1][LA + LB + 1][16][6];
    sfor<LA, LA + LB + 1>([&](auto lc) {
        constexpr int la = CV(lc);
        sfor<0, ncart(la)>([&](auto cc) { xi[0][la][CV(cc)][0] = acc[la][CV(cc)]; });
    });
    sfor<1, LB + 1>([&](auto lbc) {
        constexpr int lb = CV(lbc);
        sfor<0, ncart(lb)>([&](auto cbc) {
            constexpr int cb = CV(cbc);
            constexpr int q = dir_of(lb, cb);
            constexpr int cb1 = lower(lb, cb, q);
            sfor<LA, LA + LB - lb + 1>([&](auto lac) {
                constexpr int la = CV(lac);
                sfor<0, ncart(la)>([&](auto cac) {
                    constexpr int ca = CV(cac);
                    constexpr int ca1 = raise(la, ca, q);
                    xi[lb][la][ca][cb] = xi[lb - 1][la + 1][ca1][cb1] + AB[q] * xi[lb - 1][la][ca][cb1];
                });
            });
        });
    });
    sfor<0, ncart(LA)>([&](auto cac) {
        sfor<0, ncart(LB)>([&](auto cbc) { out[CV(cac)][CV(cbc)] = xi[LB][LA][CV(cac)][CV(cbc)]; });
    });
}

// Contracted 3c-CP block A_ab(C) of one shell pair at the lane's point C:
// Eq. vrr per primitive pair, contraction over primitives, then Eq. hrr.
template <int LA, int LB>
__device__ __forceinline__ void pair_block(const PrimPair* __restrict__ pp0, int nprim, const double (&AB)[3],
                                           double cx, double cy, double cz, const double* __restrict__ tab,
                                           double (&Ab)[ncart(LA)][ncart(LB)])
{
    constexpr int L = LA + LB;
    double acc[L + 1][16];
    sfor<LA, L + 1>([&](auto lc) {
        sfor<0, ncart(CV(lc))>([&](auto cc) { acc[CV(lc)][CV(cc)] = 0.0; });
    });
    // software pipeline: the next primitive pair's record is requested before the
    // current one is evaluated, so its scalar-load latency overlaps the arithmetic
    PrimPair nxt = pp0[0];
    for (int k = 0; k < nprim; ++k) {
        const PrimPair pp = nxt;
        if (k + 1 < nprim) nxt = pp0[k + 1];
        const double PC[3] = {pp.Px - cx, pp.Py - cy, pp.Pz - cz};
        const double PA[3] = {pp.PAx, pp.PAy, pp.PAz};
        const double T = pp.zp * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        double Fm[L + 1];
        boys<L>(T, tab, Fm);
        double th[L + 1][L + 1][16];
        sfor<0, L + 1>([&](auto nc) { th[CV(nc)][0][0] = pp.pref * Fm[CV(nc)]; });
        vrr<L>(th, PA, PC, pp.oo2zp);
        sfor<LA, L + 1>([&](auto lc) {
            sfor<0, ncart(CV(lc))>([&](auto cc) { acc[CV(lc)][CV(cc)] += th[0][CV(lc)][CV(cc)]; });
        });
    }
    hrr<LA, LB>(acc, AB, Ab);
}

template <int LA, int LB, int TA>
__global__ __launch_bounds__(256) void afg_kernel(const double* __restrict__ px, const double* __restrict__ py,
                                                  const double* __restrict__ pz, const double* __restrict__ pw,
                                                  const double* __restrict__ F, double* __restrict__ G, int64_t ld,
                                                  const PrimPair* __restrict__ prims,
                                                  const int32_t* __restrict__ runs,
                                                  const int32_t* __restrict__ btasks,
                                                  const double* __restrict__ btask_ab,
                                                  const int32_t* __restrict__ batch_run_off, int32_t nrun,
                                                  const double* __restrict__ gtab)
{
    constexpr int NA = ncart(LA), NB = ncart(LB);
    constexpr int RS = 2 + TA;        // run record stride
    constexpr int BS = 2 + 2 * TA;    // B-task record stride
    __shared__ double tab[kBoysRows * kBoysCols];
    for (int i = threadIdx.x; i < kBoysRows * kBoysCols; i += blockDim.x) tab[i] = gtab[i];
    __syncthreads();

    const int batch = blockIdx.x;
    const int64_t col = (int64_t)batch * kBatch + threadIdx.x;
    const double cx = px[col], cy = py[col], cz = pz[col], w = pw[col];

    int r0 = 0, r1 = nrun;
    if (batch_run_off) {
        r0 = batch_run_off[batch];
        r1 = batch_run_off[batch + 1];
    }
    for (int r = r0; r < r1; ++r) {
        const int32_t* run = runs + (int64_t)r * RS;
        const int b0 = run[0], b1 = run[1];
        int arow[TA];
        double Fa[TA][NA], Ga[TA][NA];
        sfor<0, TA>([&](auto kc) {
            constexpr int k = CV(kc);
            arow[k] = run[2 + k];
            sfor<0, NA>([&](auto ic) {
                constexpr int i = CV(ic);
                Fa[k][i] = arow[k] >= 0 ? cnorm(LA, i) * F[(int64_t)(arow[k] + i) * ld + col] : 0.0;
                Ga[k][i] = 0.0;
            });
        });
        // the F_B / G_B rows of the next B task are fetched one task ahead
        int nrow = 0;
        double Fn[NB], Gn[NB];
        auto fetch = [&](int bt) {
            nrow = btasks[(int64_t)bt * BS];
            sfor<0, NB>([&](auto jc) {
                const int64_t o = (int64_t)(nrow + CV(jc)) * ld + col;
                Fn[CV(jc)] = F[o];
                Gn[CV(jc)] = G[o];
            });
        };
        if (b0 < b1) fetch(b0);
        for (int bt = b0; bt < b1; ++bt) {
            const int32_t* cur = btasks + (int64_t)bt * BS;
            const int brow = nrow;
            double Fb[NB], Gold[NB], Gb[NB];
            sfor<0, NB>([&](auto jc) {
                constexpr int j = CV(jc);
                Fb[j] = cnorm(LB, j) * Fn[j];
                Gold[j] = Gn[j];
                Gb[j] = 0.0;
            });
            if (bt + 1 < b1) fetch(bt + 1);
            const int mask = cur[1];
            bool transposed = false;
            sfor<0, TA>([&](auto kc) {
                constexpr int k = CV(kc);
                if (mask & (1 << k)) {
                    const double* ab = btask_ab + ((int64_t)bt * TA + k) * 3;
                    const double AB[3] = {ab[0], ab[1], ab[2]};
                    double Ab[NA][NB];
                    pair_block<LA, LB>(prims + cur[2 + 2 * k], cur[3 + 2 * k], AB, cx, cy, cz, tab, Ab);
                    sfor<0, NA>([&](auto ic) {
                        constexpr int i = CV(ic);
                        double acc = Ga[k][i];
                        sfor<0, NB>([&](auto jc) { acc = fma(Ab[i][CV(jc)], Fb[CV(jc)], acc); });
                        Ga[k][i] = acc;
                    });
                    if (arow[k] != brow) {   // A != B: the transposed block feeds G_B
                        transposed = true;
                        sfor<0, NB>([&](auto jc) {
                            constexpr int j = CV(jc);
                            double acc = Gb[j];
                            sfor<0, NA>([&](auto ic) { acc = fma(Ab[CV(ic)][j], Fa[k][CV(ic)], acc); });
                            Gb[j] = acc;
                        });
                    }
                }
            });
            if (transposed) {
                sfor<0, NB>([&](auto jc) {
                    constexpr int j = CV(jc);
                    G[(int64_t)(brow + j) * ld + col] = fma(w * cnorm(LB, j), Gb[j], Gold[j]);
                });
            }
        }
        sfor<0, TA>([&](auto kc) {
            constexpr int k = CV(kc);
            if (arow[k] >= 0) {
                sfor<0, NA>([&](auto ic) {
                    constexpr int i = CV(ic);
                    G[(int64_t)(arow[k] + i) * ld + col] += (w * cnorm(LA, i)) * Ga[k][i];
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
    boys<MMAX>(T[k], tab, f);
    sfor<0, MMAX + 1>([&](auto mc) { F[k * (MMAX + 1) + CV(mc)] = f[CV(mc)]; });
}

}  // namespace

hipError_t launch_afg(int la, int lb, const AfgArgs& a, hipStream_t s)
{
    if (a.nbatch <= 0) return hipSuccess;
    dim3 grid(a.nbatch), block(kBatch);
#define SNK_AFG(LA, LB, TA)                                                                                    \
    hipLaunchKernelGGL((afg_kernel<LA, LB, TA>), grid, block, 0, s, a.px, a.py, a.pz, a.pw, a.F, a.G, a.ld, \
                       a.prims, a.runs, a.btasks, a.btask_ab, a.batch_run_off, a.nrun, a.boys_tab)
    switch (la * 3 + lb) {
        case 0: SNK_AFG(0, 0, kTileA[0]); break;
        case 3: SNK_AFG(1, 0, kTileA[1]); break;
        case 4: SNK_AFG(1, 1, kTileA[2]); break;
        case 6: SNK_AFG(2, 0, kTileA[3]); break;
        case 7: SNK_AFG(2, 1, kTileA[4]); break;
        case 8: SNK_AFG(2, 2, kTileA[5]); break;
        default: return hipErrorInvalidValue;
    }
#undef SNK_AFG
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
