// Density-fitted Coulomb matrix by the McMurchie-Davidson J-engine (Sec. II.B): Hermite
// densities of the orbital primitive pairs (Eq. Dp), the Coulomb potential of the density in
// the auxiliary basis (Eqs. V_df and cabP-jengine), the fitted coefficients through the
// Cholesky factor of the metric (Eq. P_df), and J in the Hermite basis of each orbital
// primitive pair, transformed back to the Cartesian pair (Eq. J_df).
//
// Work layout on gfx950: one lane per orbital primitive pair (the paper's thread per primitive
// shell), the auxiliary shells the lanes share staged through LDS or taken one per workgroup,
// so every lane of a wave runs the same recursion with no divergence; all sums are formed in a
// fixed order (no floating-point atomics), so a build is bitwise reproducible.
#include "os3c.h"

namespace snk {
namespace {

using os3c::comp;
using os3c::ncart;
using os3c::sfor;

constexpr double kTwoPi52 = 34.98683665524972;   // 2 pi^(5/2)

// Hermite components (t, u, v), t + u + v <= L: index of (t, u, v) in levels of t + u + v,
// each level in the Cartesian component order of its total
constexpr int nherm(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
constexpr int hidx(int t, int u, int v)
{
    const int L = t + u + v;
    return L * (L + 1) * (L + 2) / 6 + ((L - t) * (L - t + 1)) / 2 + v;
}
constexpr int htuv(int i, int q)
{
    int L = 0;
    while (nherm(L) <= i) ++L;
    const int c = i - (L == 0 ? 0 : nherm(L - 1));
    return comp(L, c, q);
}

// Hermite expansion coefficients of a primitive pair along one axis (McMurchie-Davidson):
// x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = sum_t E[i][j][t] Lambda_t(x_P), from
// E[0][0][0] = exp(-ab/(a+b) X_AB^2) and the two-term recursions in i and j.
template <int LA, int LB>
__device__ __forceinline__ void md_e(double a, double b, double XAB, double (&E)[LA + 1][LB + 1][LA + LB + 1])
{
    const double p = a + b, h = 0.5 / p;
    const double XPA = -b / p * XAB, XPB = a / p * XAB;
    sfor<0, LA + 1>([&](auto ic) {
        sfor<0, LB + 1>([&](auto jc) {
            constexpr int i = CV(ic), j = CV(jc);
            sfor<0, LA + LB + 1>([&](auto tc) {
                constexpr int t = CV(tc);
                double v = 0.0;
                if constexpr (i == 0 && j == 0) {
                    if constexpr (t == 0) v = exp(-a * b / p * XAB * XAB);
                } else if constexpr (t <= i + j) {
                    constexpr int i1 = i > 0 ? i - 1 : 0, j1 = i > 0 ? j : j - 1;
                    const double X = i > 0 ? XPA : XPB;
                    v = X * E[i1][j1][t];
                    if constexpr (t > 0) v += h * E[i1][j1][t - 1];
                    if constexpr (t + 1 <= i1 + j1) v += (double)(t + 1) * E[i1][j1][t + 1];
                }
                E[i][j][t] = v;
            });
        });
    });
}

// Auxiliary Hermite integrals R^0_{tuv}, t + u + v <= N (Eq. md1 with R^n_000 = (-2 alpha)^n F_n),
// one recursion level at a time from n = N down to 0.
template <int N>
__device__ __forceinline__ void md_r(double alpha, const double (&X)[3], const double (&F)[N + 1],
                                     double (&R)[nherm(N)])
{
    double lv[N + 1][nherm(N)];
    double m2a[N + 1];
    m2a[0] = 1.0;
    sfor<1, N + 1>([&](auto kc) { m2a[CV(kc)] = m2a[CV(kc) - 1] * (-2.0 * alpha); });
    sfor<0, N + 1>([&](auto kc) {
        constexpr int n = N - CV(kc);
        sfor<0, nherm(N - n)>([&](auto ic) {
            constexpr int i = CV(ic);
            constexpr int t = htuv(i, 0), u = htuv(i, 1), v = htuv(i, 2);
            double r;
            if constexpr (i == 0) {
                r = m2a[n] * F[n];
            } else if constexpr (t > 0) {
                r = X[0] * lv[n + 1][hidx(t - 1, u, v)];
                if constexpr (t > 1) r += (double)(t - 1) * lv[n + 1][hidx(t - 2, u, v)];
            } else if constexpr (u > 0) {
                r = X[1] * lv[n + 1][hidx(t, u - 1, v)];
                if constexpr (u > 1) r += (double)(u - 1) * lv[n + 1][hidx(t, u - 2, v)];
            } else {
                r = X[2] * lv[n + 1][hidx(t, u, v - 1)];
                if constexpr (v > 1) r += (double)(v - 1) * lv[n + 1][hidx(t, u, v - 2)];
            }
            lv[n][i] = r;
        });
    });
    sfor<0, nherm(N)>([&](auto ic) { R[CV(ic)] = lv[0][CV(ic)]; });
}

// (-1)^(t+u+v) of Hermite component i
template <int I>
constexpr double hsign()
{
    return ((htuv(I, 0) + htuv(I, 1) + htuv(I, 2)) & 1) ? -1.0 : 1.0;
}

template <int LP, int LC>
__device__ __forceinline__ void hermite_pair_integrals(double zp, const double (&PC)[3], double zc,
                                                       const double* __restrict__ tab, double& pref,
                                                       double (&R)[nherm(LP + LC)])
{
    constexpr int N = LP + LC;
    const double alpha = zp * zc / (zp + zc);
    const double T = alpha * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
    double F[N + 1];
    os3c::boys<N, double, kDfjBoysCols>(T, tab, F);
    md_r<N>(alpha, PC, F, R);
    pref = kTwoPi52 / (zp * zc * sqrt(zp + zc));
}

// ---------------------------------------------------------------------------------------
// Eq. Dp: D_ptilde = sum_ab E^ptilde_ab D_ab over the Cartesian components of one primitive
// pair (both orders of a shell pair A != B), one lane per primitive pair of class (LA, LB).
// ---------------------------------------------------------------------------------------
template <int LA, int LB>
__global__ __launch_bounds__(256) void hdens_kernel(const DfjPrim* __restrict__ pp, int32_t n,
                                                    const double* __restrict__ P, int64_t nbf,
                                                    double* __restrict__ Dh)
{
    constexpr int L = LA + LB;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const DfjPrim q = pp[k];
    double Ex[LA + 1][LB + 1][L + 1], Ey[LA + 1][LB + 1][L + 1], Ez[LA + 1][LB + 1][L + 1];
    md_e<LA, LB>(q.za, q.zb, q.ABx, Ex);
    md_e<LA, LB>(q.za, q.zb, q.ABy, Ey);
    md_e<LA, LB>(q.za, q.zb, q.ABz, Ez);
    double d[nherm(L)];
    sfor<0, nherm(L)>([&](auto ic) { d[CV(ic)] = 0.0; });
    sfor<0, ncart(LA)>([&](auto ac) {
        sfor<0, ncart(LB)>([&](auto bc) {
            constexpr int a = CV(ac), b = CV(bc);
            constexpr int ax = comp(LA, a, 0), ay = comp(LA, a, 1), az = comp(LA, a, 2);
            constexpr int bx = comp(LB, b, 0), by = comp(LB, b, 1), bz = comp(LB, b, 2);
            const double dab = os3c::cnorm(LA, a) * os3c::cnorm(LB, b) * P[(int64_t)(q.fa + a) * nbf + q.fb + b];
            sfor<0, ax + bx + 1>([&](auto tc) {
                sfor<0, ay + by + 1>([&](auto uc) {
                    const double exy = Ex[ax][bx][CV(tc)] * Ey[ay][by][CV(uc)] * dab;
                    sfor<0, az + bz + 1>([&](auto vc) {
                        d[hidx(CV(tc), CV(uc), CV(vc))] += exy * Ez[az][bz][CV(vc)];
                    });
                });
            });
        });
    });
    double* out = Dh + (int64_t)k * kDfjHerm;
    sfor<0, nherm(L)>([&](auto ic) { out[CV(ic)] = q.cc * d[CV(ic)]; });
}

// ---------------------------------------------------------------------------------------
// Eqs. V_df / cabP-jengine, first step: V_ctilde = sum_pairs pref sum_ptilde (ctilde|ptilde) D_ptilde
// for the auxiliary shells of angular momentum LC against one chunk of the orbital primitive
// pairs of total LP: workgroup (chunk, auxiliary shell), lane = primitive pair.  The
// workgroup's sums go to part[shell][slot] (no atomics; the slots are added in order later).
// ---------------------------------------------------------------------------------------
template <int LP, int LC>
__global__ __launch_bounds__(256) void vaux_kernel(const DfjPrim* __restrict__ pp, const double* __restrict__ Dh,
                                                   int32_t pbeg, int32_t pend, int32_t chunk, int32_t slot0,
                                                   const DfjAux* __restrict__ aux, int32_t abeg, int32_t nslot,
                                                   const double* __restrict__ gtab, double* __restrict__ part)
{
    constexpr int NC = nherm(LC), NP = nherm(LP);
    __shared__ double tab[kBoysRows * kDfjBoysCols];
    __shared__ double red[4][NC];
    for (int i = threadIdx.x; i < kBoysRows * kDfjBoysCols; i += blockDim.x) tab[i] = gtab[i];
    __syncthreads();
    const int a = abeg + blockIdx.y;
    const DfjAux c = aux[a];
    const int k0 = pbeg + blockIdx.x * chunk, k1 = min(pend, k0 + chunk);
    double acc[NC];
    sfor<0, NC>([&](auto ic) { acc[CV(ic)] = 0.0; });
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const DfjPrim q = pp[k];
        const double PC[3] = {q.Px - c.x, q.Py - c.y, q.Pz - c.z};
        double R[nherm(LP + LC)], pref;
        hermite_pair_integrals<LP, LC>(q.za + q.zb, PC, c.z_exp, tab, pref, R);
        const double* d = Dh + (int64_t)k * kDfjHerm;
        double dv[NP];
        sfor<0, NP>([&](auto ic) { dv[CV(ic)] = d[CV(ic)]; });
        sfor<0, NC>([&](auto jc) {
            constexpr int j = CV(jc);
            constexpr int tj = htuv(j, 0), uj = htuv(j, 1), vj = htuv(j, 2);
            double s = 0.0;
            sfor<0, NP>([&](auto ic) {
                constexpr int i = CV(ic);
                s += dv[i] * R[hidx(htuv(i, 0) + tj, htuv(i, 1) + uj, htuv(i, 2) + vj)];
            });
            acc[j] += hsign<j>() * pref * s;
        });
    }
    // fixed-order workgroup sum
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    sfor<0, NC>([&](auto jc) {
        double v = acc[CV(jc)];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wave][CV(jc)] = v;
    });
    __syncthreads();
    if ((int)threadIdx.x < NC) {
        const int j = threadIdx.x;
        part[((int64_t)a * nslot + slot0 + blockIdx.x) * kDfjAuxHerm + j] =
            (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
    }
}

// One-centre Hermite expansion of an auxiliary Cartesian component k (exponent z):
// x^i exp(-z x^2) = sum_t e1(i, t) Lambda_t
template <int LC>
__device__ __forceinline__ void md_e1(double z, double (&E)[LC + 1][LC + 1])
{
    double E2[LC + 1][1][LC + 1];
    md_e<LC, 0>(z, 0.0, 0.0, E2);
    sfor<0, LC + 1>([&](auto ic) { sfor<0, LC + 1>([&](auto tc) { E[CV(ic)][CV(tc)] = E2[CV(ic)][0][CV(tc)]; }); });
}

// One lane per auxiliary shell of angular momentum LC: V_ctilde summed over the slots in slot
// order, then v_k = coef cnorm_k sum_ctilde E^ctilde_k V_ctilde for its Cartesian components.
template <int LC>
__device__ __forceinline__ void vaux_finish_one(const DfjAux& c, const double* __restrict__ part, int32_t nslot,
                                                double* __restrict__ v)
{
    constexpr int NC = nherm(LC);
    double V[NC];
    sfor<0, NC>([&](auto ic) { V[CV(ic)] = 0.0; });
    for (int s = 0; s < nslot; ++s)
        sfor<0, NC>([&](auto ic) { V[CV(ic)] += part[(int64_t)s * kDfjAuxHerm + CV(ic)]; });
    double E[LC + 1][LC + 1];
    md_e1<LC>(c.z_exp, E);
    sfor<0, ncart(LC)>([&](auto kc) {
        constexpr int k = CV(kc);
        constexpr int kx = comp(LC, k, 0), ky = comp(LC, k, 1), kz = comp(LC, k, 2);
        double s = 0.0;
        sfor<0, kx + 1>([&](auto tc) {
            sfor<0, ky + 1>([&](auto uc) {
                sfor<0, kz + 1>([&](auto wc) {
                    s += E[kx][CV(tc)] * E[ky][CV(uc)] * E[kz][CV(wc)] * V[hidx(CV(tc), CV(uc), CV(wc))];
                });
            });
        });
        v[c.f0 + k] = c.coef * os3c::cnorm(LC, k) * s;
    });
}

__global__ __launch_bounds__(256) void vaux_finish_kernel(const DfjAux* __restrict__ aux, int32_t naux,
                                                          const double* __restrict__ part, int32_t nslot,
                                                          double* __restrict__ v)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= naux) return;
    const DfjAux c = aux[a];
    const double* p = part + (int64_t)a * nslot * kDfjAuxHerm;
    if (c.l == 0) vaux_finish_one<0>(c, p, nslot, v);
    else if (c.l == 1) vaux_finish_one<1>(c, p, nslot, v);
    else vaux_finish_one<2>(c, p, nslot, v);
}

// Hermite density of each auxiliary shell from the fitted coefficients d:
// D_ctilde = coef sum_k cnorm_k E^ctilde_k d_k (the auxiliary analogue of Eq. Dp)
template <int LC>
__device__ __forceinline__ void auxdens_one(const DfjAux& c, const double* __restrict__ d, double* __restrict__ out)
{
    constexpr int NC = nherm(LC);
    double E[LC + 1][LC + 1];
    md_e1<LC>(c.z_exp, E);
    double D[NC];
    sfor<0, NC>([&](auto ic) { D[CV(ic)] = 0.0; });
    sfor<0, ncart(LC)>([&](auto kc) {
        constexpr int k = CV(kc);
        constexpr int kx = comp(LC, k, 0), ky = comp(LC, k, 1), kz = comp(LC, k, 2);
        const double dk = c.coef * os3c::cnorm(LC, k) * d[c.f0 + k];
        sfor<0, kx + 1>([&](auto tc) {
            sfor<0, ky + 1>([&](auto uc) {
                sfor<0, kz + 1>([&](auto wc) {
                    D[hidx(CV(tc), CV(uc), CV(wc))] += E[kx][CV(tc)] * E[ky][CV(uc)] * E[kz][CV(wc)] * dk;
                });
            });
        });
    });
    sfor<0, kDfjAuxHerm>([&](auto ic) {
        constexpr int i = CV(ic);
        if constexpr (i < NC) out[i] = D[i];
        else out[i] = 0.0;
    });
}

__global__ __launch_bounds__(256) void auxdens_kernel(const DfjAux* __restrict__ aux, int32_t naux,
                                                      const double* __restrict__ d, double* __restrict__ Dc)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= naux) return;
    const DfjAux c = aux[a];
    double* out = Dc + (int64_t)a * kDfjAuxHerm;
    if (c.l == 0) auxdens_one<0>(c, d, out);
    else if (c.l == 1) auxdens_one<1>(c, d, out);
    else auxdens_one<2>(c, d, out);
}

// ---------------------------------------------------------------------------------------
// Eq. J_df in the Hermite basis: J_ptilde = sum_c pref sum_ctilde (ptilde|ctilde) D_ctilde over
// every auxiliary shell, then J_ab = cc sum_ptilde E^ptilde_ab J_ptilde for the Cartesian
// components of the lane's primitive pair (class (LA, LB)); the auxiliary shells (ordered by
// angular momentum) are staged through LDS in blocks shared by the workgroup.
// ---------------------------------------------------------------------------------------
constexpr int kAuxBlock = 128;

template <int LP, int LC>
__device__ __forceinline__ void jp_accumulate(double zp, const double (&P)[3], const DfjAux& c,
                                              const double* __restrict__ Dc, const double* __restrict__ tab,
                                              double (&J)[nherm(LP)])
{
    constexpr int NC = nherm(LC);
    const double PC[3] = {P[0] - c.x, P[1] - c.y, P[2] - c.z};
    double R[nherm(LP + LC)], pref;
    hermite_pair_integrals<LP, LC>(zp, PC, c.z_exp, tab, pref, R);
    sfor<0, nherm(LP)>([&](auto ic) {
        constexpr int i = CV(ic);
        double s = 0.0;
        sfor<0, NC>([&](auto jc) {
            constexpr int j = CV(jc);
            s += hsign<j>() * Dc[j] *
                 R[hidx(htuv(i, 0) + htuv(j, 0), htuv(i, 1) + htuv(j, 1), htuv(i, 2) + htuv(j, 2))];
        });
        J[i] += pref * s;
    });
}

// Eq. J_df in the Hermite basis: one lane per orbital primitive pair p, J_p~ = sum over the
// auxiliary shells c of workgroup row blockIdx.y (shells [y chunk, (y + 1) chunk)) of
// sum_c~ (p~|c~) D_c~, the shells staged through LDS in blocks of kAuxBlock.  Splitting the
// auxiliary shells over workgroup rows fills the device when the orbital pairs are few; the
// rows' sums go to Jh[y][p][p~] and jpair_finish_kernel adds them in row order.
template <int LA, int LB>
__global__ __launch_bounds__(256) void jpair_kernel(const DfjPrim* __restrict__ pp, int32_t n,
                                                    const DfjAux* __restrict__ aux, const double* __restrict__ Dc,
                                                    const int32_t* __restrict__ lbeg,   // [4] aux ranges by l
                                                    const double* __restrict__ gtab, int32_t chunk,
                                                    double* __restrict__ Jh)
{
    constexpr int LP = LA + LB;
    constexpr int NH = nherm(LP);
    __shared__ double tab[kBoysRows * kDfjBoysCols];
    __shared__ DfjAux sa[kAuxBlock];
    __shared__ double sd[kAuxBlock][kDfjAuxHerm];
    for (int i = threadIdx.x; i < kBoysRows * kDfjBoysCols; i += blockDim.x) tab[i] = gtab[i];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = k < n;
    const DfjPrim q = pp[live ? k : 0];
    const double P[3] = {q.Px, q.Py, q.Pz};
    const double zp = q.za + q.zb;
    double J[NH];
    sfor<0, NH>([&](auto ic) { J[CV(ic)] = 0.0; });
    const int a_beg = blockIdx.y * chunk, a_end = min(lbeg[3], a_beg + chunk);
    for (int b0 = a_beg; b0 < a_end; b0 += kAuxBlock) {
        const int nb = min(kAuxBlock, a_end - b0);
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x) sa[i] = aux[b0 + i];
        for (int i = threadIdx.x; i < nb * kDfjAuxHerm; i += blockDim.x)
            sd[i / kDfjAuxHerm][i % kDfjAuxHerm] = Dc[(int64_t)b0 * kDfjAuxHerm + i];
        __syncthreads();
        // the three angular-momentum ranges of the block, in order
        for (int i = max(b0, lbeg[0]); i < min(b0 + nb, lbeg[1]); ++i)
            jp_accumulate<LP, 0>(zp, P, sa[i - b0], sd[i - b0], tab, J);
        for (int i = max(b0, lbeg[1]); i < min(b0 + nb, lbeg[2]); ++i)
            jp_accumulate<LP, 1>(zp, P, sa[i - b0], sd[i - b0], tab, J);
        for (int i = max(b0, lbeg[2]); i < min(b0 + nb, lbeg[3]); ++i)
            jp_accumulate<LP, 2>(zp, P, sa[i - b0], sd[i - b0], tab, J);
    }
    if (!live) return;
    double* out = Jh + ((int64_t)blockIdx.y * n + k) * NH;
    sfor<0, NH>([&](auto ic) { out[CV(ic)] = J[CV(ic)]; });
}

// One lane per orbital primitive pair: J_p~ summed over the nchunk rows of jpair_kernel in
// order, then taken back to the Cartesian pair (Eq. Dp in reverse) and scaled.
template <int LA, int LB>
__global__ __launch_bounds__(256) void jpair_finish_kernel(const DfjPrim* __restrict__ pp, int32_t n,
                                                           const double* __restrict__ Jh, int32_t nchunk,
                                                           double* __restrict__ Jpp)
{
    constexpr int LP = LA + LB;
    constexpr int NH = nherm(LP);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const DfjPrim q = pp[k];
    double J[NH];
    sfor<0, NH>([&](auto ic) { J[CV(ic)] = Jh[(int64_t)k * NH + CV(ic)]; });
    for (int c = 1; c < nchunk; ++c) {
        const double* in = Jh + ((int64_t)c * n + k) * NH;
        sfor<0, NH>([&](auto ic) { J[CV(ic)] += in[CV(ic)]; });
    }
    double Ex[LA + 1][LB + 1][LP + 1], Ey[LA + 1][LB + 1][LP + 1], Ez[LA + 1][LB + 1][LP + 1];
    md_e<LA, LB>(q.za, q.zb, q.ABx, Ex);
    md_e<LA, LB>(q.za, q.zb, q.ABy, Ey);
    md_e<LA, LB>(q.za, q.zb, q.ABz, Ez);
    double* out = Jpp + (int64_t)k * kDfjCart;
    sfor<0, ncart(LA)>([&](auto ac) {
        sfor<0, ncart(LB)>([&](auto bc) {
            constexpr int a = CV(ac), b = CV(bc);
            constexpr int ax = comp(LA, a, 0), ay = comp(LA, a, 1), az = comp(LA, a, 2);
            constexpr int bx = comp(LB, b, 0), by = comp(LB, b, 1), bz = comp(LB, b, 2);
            double s = 0.0;
            sfor<0, ax + bx + 1>([&](auto tc) {
                sfor<0, ay + by + 1>([&](auto uc) {
                    sfor<0, az + bz + 1>([&](auto vc) {
                        s += Ex[ax][bx][CV(tc)] * Ey[ay][by][CV(uc)] * Ez[az][bz][CV(vc)] *
                             J[hidx(CV(tc), CV(uc), CV(vc))];
                    });
                });
            });
            out[a * ncart(LB) + b] = q.cc1 * os3c::cnorm(LA, a) * os3c::cnorm(LB, b) * s;
        });
    });
}

// One lane per orbital shell pair: its primitive pairs' blocks summed in order, written to
// J[A][B] and, for A != B, to J[B][A].
__global__ __launch_bounds__(256) void jcollect_kernel(const DfjShellPair* __restrict__ sp, int32_t nsp,
                                                       const double* __restrict__ Jpp, double* __restrict__ J,
                                                       int64_t nbf)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsp) return;
    const DfjShellPair s = sp[k];
    const int na = (s.la + 1) * (s.la + 2) / 2, nb = (s.lb + 1) * (s.lb + 2) / 2;
    for (int e = 0; e < na * nb; ++e) {
        double v = 0.0;
        for (int p = s.pbeg; p < s.pbeg + s.np; ++p) v += Jpp[(int64_t)p * kDfjCart + e];
        const int ia = e / nb, ib = e - ia * nb;
        J[(int64_t)(s.fa + ia) * nbf + s.fb + ib] = v;
        if (s.fa != s.fb) J[(int64_t)(s.fb + ib) * nbf + s.fa + ia] = v;
    }
}

// ---------------------------------------------------------------------------------------
// Metric V_KL = (K|L) (set-up): one lane per auxiliary shell pair K >= L.
// ---------------------------------------------------------------------------------------
template <int LK, int LL>
__device__ __forceinline__ void metric_block(const DfjAux& K, const DfjAux& L, const double* __restrict__ tab,
                                             double* __restrict__ V, int64_t n)
{
    const double KL[3] = {K.x - L.x, K.y - L.y, K.z - L.z};
    double R[nherm(LK + LL)], pref;
    hermite_pair_integrals<LK, LL>(K.z_exp, KL, L.z_exp, tab, pref, R);
    double EK[LK + 1][LK + 1], EL[LL + 1][LL + 1];
    md_e1<LK>(K.z_exp, EK);
    md_e1<LL>(L.z_exp, EL);
    sfor<0, ncart(LK)>([&](auto kc) {
        sfor<0, ncart(LL)>([&](auto lc) {
            constexpr int k = CV(kc), l = CV(lc);
            constexpr int kx = comp(LK, k, 0), ky = comp(LK, k, 1), kz = comp(LK, k, 2);
            constexpr int lx = comp(LL, l, 0), ly = comp(LL, l, 1), lz = comp(LL, l, 2);
            double s = 0.0;
            sfor<0, kx + 1>([&](auto t1) {
                sfor<0, ky + 1>([&](auto u1) {
                    sfor<0, kz + 1>([&](auto v1) {
                        const double ek = EK[kx][CV(t1)] * EK[ky][CV(u1)] * EK[kz][CV(v1)];
                        sfor<0, lx + 1>([&](auto t2) {
                            sfor<0, ly + 1>([&](auto u2) {
                                sfor<0, lz + 1>([&](auto v2) {
                                    constexpr int sg = (CV(t2) + CV(u2) + CV(v2)) & 1;
                                    const double el = EL[lx][CV(t2)] * EL[ly][CV(u2)] * EL[lz][CV(v2)];
                                    const double r = R[hidx(CV(t1) + CV(t2), CV(u1) + CV(u2), CV(v1) + CV(v2))];
                                    s += (sg ? -1.0 : 1.0) * ek * el * r;
                                });
                            });
                        });
                    });
                });
            });
            const double val = pref * K.coef * L.coef * os3c::cnorm(LK, k) * os3c::cnorm(LL, l) * s;
            V[(int64_t)(K.f0 + k) * n + L.f0 + l] = val;
            V[(int64_t)(L.f0 + l) * n + K.f0 + k] = val;
        });
    });
}

__global__ __launch_bounds__(256) void metric_kernel(const DfjAux* __restrict__ aux, int32_t naux,
                                                     const double* __restrict__ gtab, double* __restrict__ V,
                                                     int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)naux * (naux + 1) / 2) return;
    int i = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while ((int64_t)i * (i + 1) / 2 > q) --i;
    while ((int64_t)(i + 1) * (i + 2) / 2 <= q) ++i;
    const int j = (int)(q - (int64_t)i * (i + 1) / 2);
    const DfjAux K = aux[i], L = aux[j];
    const double* tab = gtab;
#define SNK_MB(a, b) metric_block<a, b>(K, L, tab, V, n)
    if (K.l == 0) {
        if (L.l == 0) SNK_MB(0, 0);
        else if (L.l == 1) SNK_MB(0, 1);
        else SNK_MB(0, 2);
    } else if (K.l == 1) {
        if (L.l == 0) SNK_MB(1, 0);
        else if (L.l == 1) SNK_MB(1, 1);
        else SNK_MB(1, 2);
    } else {
        if (L.l == 0) SNK_MB(2, 0);
        else if (L.l == 1) SNK_MB(2, 1);
        else SNK_MB(2, 2);
    }
#undef SNK_MB
}

// ---------------------------------------------------------------------------------------
// Cholesky factorisation of the metric (set-up), blocked by kCholB columns: the diagonal
// block in LDS, the panel below it by substitution, the trailing lower triangle updated.
// A is n x n row-major; on return its lower triangle holds L (A = L L^T).
// ---------------------------------------------------------------------------------------
constexpr int kCholB = 32;

__global__ __launch_bounds__(256) void chol_diag_kernel(double* __restrict__ A, int64_t n, int64_t j0,
                                                        int32_t* __restrict__ status)
{
    __shared__ double L[kCholB][kCholB + 1];
    const int nb = (int)min<int64_t>(kCholB, n - j0);
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) L[e / nb][e % nb] = A[(j0 + e / nb) * n + j0 + e % nb];
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (threadIdx.x == 0) {
            const double d = L[k][k];
            if (!(d > 0.0)) *status = 1;   // not positive definite
            L[k][k] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        for (int i = k + 1 + threadIdx.x; i < nb; i += blockDim.x) L[i][k] /= L[k][k];
        __syncthreads();
        for (int e = threadIdx.x; e < (nb - k - 1) * (nb - k - 1); e += blockDim.x) {
            const int i = k + 1 + e / (nb - k - 1), j = k + 1 + e % (nb - k - 1);
            if (j <= i) L[i][j] -= L[i][k] * L[j][k];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e % nb;
        A[(j0 + i) * n + j0 + j] = j <= i ? L[i][j] : 0.0;
    }
}

// rows i >= j0 + kCholB: L21 = A21 L11^-T, one lane per row
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int64_t n, int64_t j0)
{
    __shared__ double L[kCholB][kCholB + 1];
    for (int e = threadIdx.x; e < kCholB * kCholB; e += blockDim.x)
        L[e / kCholB][e % kCholB] = A[(j0 + e / kCholB) * n + j0 + e % kCholB];
    __syncthreads();
    const int64_t i = j0 + kCholB + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* row = A + i * n + j0;
    double x[kCholB];
#pragma unroll
    for (int j = 0; j < kCholB; ++j) {
        double s = row[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= x[k] * L[j][k];
        x[j] = s / L[j][j];
    }
#pragma unroll
    for (int j = 0; j < kCholB; ++j) row[j] = x[j];
}

// trailing update of the lower triangle: A[i][j] -= sum_k L21[i][k] L21[j][k] for i >= j >= j0 + kCholB,
// one workgroup per kCholB x kCholB block (bi >= bj), both panels staged in LDS
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int64_t n, int64_t j0)
{
    __shared__ double Pi[kCholB][kCholB + 1];
    __shared__ double Pj[kCholB][kCholB + 1];
    const int64_t nbk = (n - j0 - kCholB + kCholB - 1) / kCholB;
    // block index -> (bi, bj), bi >= bj
    const int64_t q = blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > q) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
    const int64_t bj = q - bi * (bi + 1) / 2;
    if (bi >= nbk) return;
    const int64_t r0 = j0 + kCholB + bi * kCholB, c0 = j0 + kCholB + bj * kCholB;
    for (int e = threadIdx.x; e < kCholB * kCholB; e += blockDim.x) {
        const int r = e / kCholB, k = e % kCholB;
        Pi[r][k] = r0 + r < n ? A[(r0 + r) * n + j0 + k] : 0.0;
        Pj[r][k] = c0 + r < n ? A[(c0 + r) * n + j0 + k] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCholB * kCholB; e += blockDim.x) {
        const int r = e / kCholB, c = e % kCholB;
        const int64_t i = r0 + r, j = c0 + c;
        if (i >= n || j >= n || j > i) continue;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < kCholB; ++k) s += Pi[r][k] * Pj[c][k];
        A[i * n + j] -= s;
    }
}

// Eq. P_df at set-up: L^-1 column by column.  Workgroup j solves L x = e_j by forward
// substitution in blocks of 64 unknowns (the sixteen waves form the block rows' dot products
// with the unknowns already solved, lanes along the row with a fixed-order wave sum; one wave
// solves the block's triangle from LDS, lane r holding unknown r) and writes x as row j of
// W = L^-T (W[j][i] = (L^-1)_ij, zero for i < j).
constexpr int kSolveB = 64;

constexpr int kSolveThreads = 1024;   // sixteen waves keep the row loads of a block in flight

__global__ __launch_bounds__(kSolveThreads) void tri_inverse_kernel(const double* __restrict__ L, int64_t n,
                                                                    double* __restrict__ W)
{
    __shared__ double blk[kSolveB][kSolveB + 1];
    __shared__ double part[kSolveB];
    const int64_t j = blockIdx.x;
    double* x = W + j * n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t jb = (j / kSolveB) * kSolveB;   // the block holding unknown j
    for (int64_t i = tid; i < jb; i += blockDim.x) x[i] = 0.0;
    for (int64_t b0 = jb; b0 < n; b0 += kSolveB) {
        const int nb = (int)min<int64_t>(kSolveB, n - b0);
        for (int r = wave; r < nb; r += kSolveThreads / 64) {
            const double* row = L + (b0 + r) * n;
            double s = 0.0;
#pragma unroll 4
            for (int64_t k = jb + lane; k < b0; k += 64) s += row[k] * x[k];
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
            if (lane == 0) part[r] = s;
        }
        for (int e = tid; e < nb * nb; e += blockDim.x) blk[e / nb][e % nb] = L[(b0 + e / nb) * n + b0 + e % nb];
        __syncthreads();
        if (wave == 0) {
            double xv = lane < nb ? (b0 + lane == j ? 1.0 : 0.0) - part[lane] : 0.0;
            for (int c = 0; c < nb; ++c) {
                const double xc = __shfl(xv, c) / blk[c][c];
                if (lane == c) xv = xc;
                else if (lane > c && lane < nb) xv -= blk[lane][c] * xc;
            }
            if (lane < nb) x[b0 + lane] = xv;
        }
        __syncthreads();
    }
}

// out = in^T (n x n)
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ in, int64_t n,
                                                        double* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e - i * n;
    out[e] = in[j * n + i];
}

// Eq. P_df per build: y_i = sum_k M_ik x_k over k <= i (lower) or k >= i (upper); one wave per
// row, lanes along the row, fixed-order sums.
__global__ __launch_bounds__(256) void trmv_kernel(const double* __restrict__ M, int64_t n,
                                                   const double* __restrict__ x, double* __restrict__ y, int lower)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const double* row = M + i * n;
    const int64_t k0 = lower ? 0 : i, k1 = lower ? i + 1 : n;
    double s = 0.0;
#pragma unroll 4
    for (int64_t k = k0 + lane; k < k1; k += 64) s += row[k] * x[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[i] = s;
}

__global__ __launch_bounds__(256) void dot_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* __restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += a[i] * b[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

hipError_t launch_dfj_hdens(int cls, const DfjPrim* pp, int32_t n, const double* P, int64_t nbf, double* Dh,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    switch (cls) {
        case 0: hipLaunchKernelGGL((hdens_kernel<0, 0>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        case 1: hipLaunchKernelGGL((hdens_kernel<1, 0>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        case 2: hipLaunchKernelGGL((hdens_kernel<1, 1>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        case 3: hipLaunchKernelGGL((hdens_kernel<2, 0>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        case 4: hipLaunchKernelGGL((hdens_kernel<2, 1>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        case 5: hipLaunchKernelGGL((hdens_kernel<2, 2>), g, b, 0, s, pp, n, P, nbf, Dh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dfj_vaux(int LP, int LC, const DfjPrim* pp, const double* Dh, int32_t pbeg, int32_t pend,
                           int32_t chunk, int32_t slot0, const DfjAux* aux, int32_t abeg, int32_t aend, int32_t nslot,
                           const double* tab, double* part, hipStream_t s)
{
    if (pend <= pbeg || aend <= abeg) return hipSuccess;
    const dim3 g((pend - pbeg + chunk - 1) / chunk, aend - abeg), b(256);
#define SNK_V(P_, C_)                                                                                          \
    if (LP == P_ && LC == C_) {                                                                                \
        hipLaunchKernelGGL((vaux_kernel<P_, C_>), g, b, 0, s, pp, Dh, pbeg, pend, chunk, slot0, aux, abeg,    \
                           nslot, tab, part);                                                                  \
        return hipGetLastError();                                                                              \
    }
    SNK_V(0, 0) SNK_V(0, 1) SNK_V(0, 2) SNK_V(1, 0) SNK_V(1, 1) SNK_V(1, 2) SNK_V(2, 0) SNK_V(2, 1) SNK_V(2, 2)
    SNK_V(3, 0) SNK_V(3, 1) SNK_V(3, 2) SNK_V(4, 0) SNK_V(4, 1) SNK_V(4, 2)
#undef SNK_V
    return hipErrorInvalidValue;
}

hipError_t launch_dfj_vfinish(const DfjAux* aux, int32_t naux, const double* part, int32_t nslot, double* v,
                              hipStream_t s)
{
    if (naux <= 0) return hipSuccess;
    hipLaunchKernelGGL(vaux_finish_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, aux, naux, part, nslot, v);
    return hipGetLastError();
}

hipError_t launch_dfj_auxdens(const DfjAux* aux, int32_t naux, const double* d, double* Dc, hipStream_t s)
{
    if (naux <= 0) return hipSuccess;
    hipLaunchKernelGGL(auxdens_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, aux, naux, d, Dc);
    return hipGetLastError();
}

int dfj_jpair_chunks(int32_t n, int32_t naux)
{
    // about 2048 workgroups per class, each row of them at least kAuxBlock / 4 shells
    const int64_t wg = std::max<int64_t>(1, (n + 255) / 256);
    const int64_t want = std::max<int64_t>(1, 2048 / wg);
    const int64_t most = std::max<int64_t>(1, naux / (kAuxBlock / 4));
    return (int)std::min<int64_t>(want, most);
}

hipError_t launch_dfj_jpair(int cls, const DfjPrim* pp, int32_t n, const DfjAux* aux, int32_t naux, const double* Dc,
                            const int32_t* lbeg, const double* tab, double* Jh, double* Jpp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int nchunk = dfj_jpair_chunks(n, naux);
    const int chunk = (naux + nchunk - 1) / nchunk;
    const dim3 g((n + 255) / 256, nchunk), gf((n + 255) / 256), b(256);
#define SNK_JP(LA, LB)                                                                                          \
    hipLaunchKernelGGL((jpair_kernel<LA, LB>), g, b, 0, s, pp, n, aux, Dc, lbeg, tab, chunk, Jh);                \
    hipLaunchKernelGGL((jpair_finish_kernel<LA, LB>), gf, b, 0, s, pp, n, Jh, nchunk, Jpp)
    switch (cls) {
        case 0: SNK_JP(0, 0); break;
        case 1: SNK_JP(1, 0); break;
        case 2: SNK_JP(1, 1); break;
        case 3: SNK_JP(2, 0); break;
        case 4: SNK_JP(2, 1); break;
        case 5: SNK_JP(2, 2); break;
        default: return hipErrorInvalidValue;
    }
#undef SNK_JP
    return hipGetLastError();
}

hipError_t launch_dfj_jcollect(const DfjShellPair* sp, int32_t nsp, const double* Jpp, double* J, int64_t nbf,
                               hipStream_t s)
{
    if (nsp <= 0) return hipSuccess;
    hipLaunchKernelGGL(jcollect_kernel, dim3((nsp + 255) / 256), dim3(256), 0, s, sp, nsp, Jpp, J, nbf);
    return hipGetLastError();
}

hipError_t launch_dfj_metric(const DfjAux* aux, int32_t naux, const double* tab, double* V, int64_t n, hipStream_t s)
{
    const int64_t np = (int64_t)naux * (naux + 1) / 2;
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(metric_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, aux, naux, tab, V, n);
    return hipGetLastError();
}

hipError_t launch_dfj_cholesky(double* A, int64_t n, int32_t* status, hipStream_t s)
{
    for (int64_t j0 = 0; j0 < n; j0 += kCholB) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, A, n, j0, status);
        const int64_t rest = n - j0 - kCholB;
        if (rest > 0) {
            hipLaunchKernelGGL(chol_panel_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, A, n, j0);
            const int64_t nbk = (rest + kCholB - 1) / kCholB;
            hipLaunchKernelGGL(chol_update_kernel, dim3((unsigned)(nbk * (nbk + 1) / 2)), dim3(256), 0, s, A, n, j0);
        }
    }
    return hipGetLastError();
}

hipError_t launch_dfj_invert(double* L, int64_t n, double* W, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(tri_inverse_kernel, dim3((unsigned)n), dim3(kSolveThreads), 0, s, L, n, W);
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, W, n, L);
    return hipGetLastError();
}

hipError_t launch_dfj_solve(const double* Linv, const double* W, int64_t n, const double* v, double* y, double* d,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 3) / 4));
    hipLaunchKernelGGL(trmv_kernel, grid, dim3(256), 0, s, Linv, n, v, y, 1);
    hipLaunchKernelGGL(trmv_kernel, grid, dim3(256), 0, s, W, n, y, d, 0);
    return hipGetLastError();
}

hipError_t launch_dfj_dot(const double* a, const double* b, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

}  // namespace snk
