// Device building blocks of the 3c-CP integrals (App. A), shared by the A.F digestion
// kernels and the screening kernels: Cartesian component tables, the Boys function
// (Eq. boys), the vertical and horizontal Obara-Saika recursions (Eqs. vrr, hrr) and the
// contracted block of one shell pair at one grid point.
#pragma once

#include "snk_internal.h"

#include <type_traits>

namespace snk {
namespace os3c {

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
// above: F_0 = sqrt(pi/T)/2, F_m = F_{m-1} (2m-1)/(2T).  R = double uses kBoysTerms
// terms; R = float (reduced-precision blocks) uses 7, whose truncation error
// (1/8)^7 / 7! ~ 1e-10 is far below FP32 rounding.
template <typename R>
constexpr int boys_terms() { return std::is_same<R, double>::value ? kBoysTerms : 7; }

// TC: columns per row of the table in memory (kBoysCols for the tables of the 3c-CP kernels,
// more for higher orders, or a prefix of at least L + boys_terms<R>() columns)
template <int L, typename R, int TC = kBoysCols>
__device__ __forceinline__ void boys(R T, const R* __restrict__ tab, R (&F)[L + 1])
{
    constexpr int NT = boys_terms<R>();
    if (T < (R)kBoysTmax) {
        const int k = (int)(T * (R)(1.0 / kBoysStep) + (R)0.5);
        const R d = (R)k * (R)kBoysStep - T;
        static_assert(TC >= L + NT, "Boys table too narrow");
        const R* row = tab + k * TC;
        R pw[NT];
        pw[0] = (R)1;
        sfor<1, NT>([&](auto jc) {
            constexpr int j = CV(jc);
            pw[j] = pw[j - 1] * (d * (R)(1.0 / j));
        });
        sfor<0, L + 1>([&](auto mc) {
            constexpr int m = CV(mc);
            R s = row[m + NT - 1] * pw[NT - 1];
            sfor<0, NT - 1>([&](auto jc) {
                constexpr int j = NT - 2 - CV(jc);
                s = fma(row[m + j], pw[j], s);
            });
            F[m] = s;
        });
    } else {
        const R r = rsqrt(T);
        const R h = (R)0.5 * r * r;
        F[0] = (R)0.88622692545275801365 * r;
        sfor<1, L + 1>([&](auto mc) {
            constexpr int m = CV(mc);
            F[m] = F[m - 1] * ((R)(2 * m - 1) * h);
        });
    }
}

// Eq. vrr: Theta^n_{a+1q} = PA_q Theta^n_a - PC_q Theta^{n+1}_a + a_q/(2 zeta_p) (Theta^n_{a-1q} - Theta^{n+1}_{a-1q})
template <int L, typename R>
__device__ __forceinline__ void vrr(R (&th)[L + 1][L + 1][16], const R (&PA)[3], const R (&PC)[3], R oo2zp)
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
                R v = PA[q] * th[n][l - 1][c1] - PC[q] * th[n + 1][l - 1][c1];
                if constexpr (am > 0) v += ((R)am * oo2zp) * (th[n][l - 2][c2] - th[n + 1][l - 2][c2]);
                th[n][l][c] = v;
            });
        });
    });
}

// Eq. hrr: Xi_{a(b+1q)} = Xi_{(a+1q)b} + AB_q Xi_{ab}, from Xi_{a0} = contracted Theta^0_a
template <int LA, int LB, typename R>
__device__ __forceinline__ void hrr(const R (&acc)[LA + LB + 1][16], const R (&AB)[3], R (&out)[ncart(LA)][ncart(LB)])
{
    R xi[LB + 1][LA + LB + 1][16][6];
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

// primitive-pair record of the arithmetic type
template <typename R>
struct PrimOf;
template <>
struct PrimOf<double> {
    typedef PrimPair type;
};
template <>
struct PrimOf<float> {
    typedef PrimPair32 type;
};

// Contracted 3c-CP blocks A_ab(C_p) of one shell pair at the lane's NP points C_p:
// Eq. vrr per primitive pair and point, contraction over primitives, then Eq. hrr.  Each
// primitive-pair record is loaded once for all NP points.
template <int LA, int LB, typename R, int NP, int TC = kBoysCols>
__device__ __forceinline__ void pair_block_n(const typename PrimOf<R>::type* __restrict__ pp0, int nprim,
                                             const R (&AB)[3], const R (&cx)[NP], const R (&cy)[NP],
                                             const R (&cz)[NP], const R* __restrict__ tab,
                                             R (&Ab)[NP][ncart(LA)][ncart(LB)])
{
    typedef typename PrimOf<R>::type PP;
    constexpr int L = LA + LB;
    R acc[NP][L + 1][16];
    sfor<0, NP>([&](auto pc) {
        sfor<LA, L + 1>([&](auto lc) {
            sfor<0, ncart(CV(lc))>([&](auto cc) { acc[CV(pc)][CV(lc)][CV(cc)] = (R)0; });
        });
    });
    auto prim = [&](const PP& pp) {
        const R PA[3] = {pp.PAx, pp.PAy, pp.PAz};
        sfor<0, NP>([&](auto pc) {
            constexpr int p = CV(pc);
            const R PC[3] = {pp.Px - cx[p], pp.Py - cy[p], pp.Pz - cz[p]};
            const R T = pp.zp * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
            R Fm[L + 1];
            boys<L, R, TC>(T, tab, Fm);
            R th[L + 1][L + 1][16];
            sfor<0, L + 1>([&](auto nc) { th[CV(nc)][0][0] = pp.pref * Fm[CV(nc)]; });
            vrr<L, R>(th, PA, PC, pp.oo2zp);
            sfor<LA, L + 1>([&](auto lc) {
                sfor<0, ncart(CV(lc))>([&](auto cc) { acc[p][CV(lc)][CV(cc)] += th[0][CV(lc)][CV(cc)]; });
            });
        });
    };
    // software pipeline: the next primitive pair's record is requested before the
    // current one is evaluated, so its scalar-load latency overlaps the arithmetic
    PP nxt{};
    if (nprim > 0) nxt = pp0[0];
    for (int k = 0; k < nprim; ++k) {
        const PP pp = nxt;
        if (k + 1 < nprim) nxt = pp0[k + 1];
        prim(pp);
    }
    sfor<0, NP>([&](auto pc) { hrr<LA, LB, R>(acc[CV(pc)], AB, Ab[CV(pc)]); });
}

// One point: A_ab(C) of one shell pair at the lane's point C.
template <int LA, int LB, typename R>
__device__ __forceinline__ void pair_block(const typename PrimOf<R>::type* __restrict__ pp0, int nprim,
                                           const R (&AB)[3], R cx, R cy, R cz, const R* __restrict__ tab,
                                           R (&Ab)[ncart(LA)][ncart(LB)])
{
    const R x[1] = {cx}, y[1] = {cy}, z[1] = {cz};
    R out[1][ncart(LA)][ncart(LB)];
    pair_block_n<LA, LB, R, 1>(pp0, nprim, AB, x, y, z, tab, out);
    sfor<0, ncart(LA)>([&](auto ic) {
        sfor<0, ncart(LB)>([&](auto jc) { Ab[CV(ic)][CV(jc)] = out[0][CV(ic)][CV(jc)]; });
    });
}

// Eq. vrr for a same-centre primitive pair (R_p = R_A, so PA = 0 and its term drops)
template <int L, typename R>
__device__ __forceinline__ void vrr_same_centre(R (&th)[L + 1][L + 1][16], const R (&PC)[3], R oo2zp)
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
                R v = -PC[q] * th[n + 1][l - 1][c1];
                if constexpr (am > 0) v += ((R)am * oo2zp) * (th[n][l - 2][c2] - th[n + 1][l - 2][c2]);
                th[n][l][c] = v;
            });
        });
    });
}

// Diagonal A_cc(C) of the contracted same-shell block (A, A) at the lane's point, from
// same-centre primitive-pair records (P = R_A).  With R_AB = 0 Eq. hrr only moves exponents
// from b onto a, so A_cc is the contracted Theta^0 of the level-2L component with exponents
// 2c; the recursion keeps only the entries those components need.
template <int L, typename R, int TC = kBoysCols>
__device__ __forceinline__ void diag_block(const typename PrimOf<R>::type* __restrict__ pp0, int nprim, R cx, R cy,
                                           R cz, const R* __restrict__ tab, R (&Acc)[ncart(L)])
{
    typedef typename PrimOf<R>::type PP;
    constexpr int L2 = 2 * L;
    sfor<0, ncart(L)>([&](auto cc) { Acc[CV(cc)] = (R)0; });
    auto prim = [&](const PP& pp) {
        const R PC[3] = {pp.Px - cx, pp.Py - cy, pp.Pz - cz};
        const R T = pp.zp * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        R Fm[L2 + 1];
        boys<L2, R, TC>(T, tab, Fm);
        R th[L2 + 1][L2 + 1][16];
        sfor<0, L2 + 1>([&](auto nc) { th[CV(nc)][0][0] = pp.pref * Fm[CV(nc)]; });
        vrr_same_centre<L2, R>(th, PC, pp.oo2zp);
        sfor<0, ncart(L)>([&](auto cc) {
            constexpr int c = CV(cc);
            Acc[c] += th[0][L2][cidx(L2, 2 * comp(L, c, 0), 2 * comp(L, c, 2))];
        });
    };
    PP nxt{};
    if (nprim > 0) nxt = pp0[0];
    for (int k = 0; k < nprim; ++k) {
        const PP pp = nxt;
        if (k + 1 < nprim) nxt = pp0[k + 1];
        prim(pp);
    }
}

}  // namespace os3c
}  // namespace snk
