/*
 * CPU FP64 oracle for the seminumerical exact-exchange (sn-K) build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the sn-K result for a given
 * basis, grid and density (Sec. II.D):
 *   Phi_{mu i}  = phi_mu(r_i)                               (Eq. collocation)
 *   F_{lam i}   = sum_nu P_{lam nu} Phi_{nu i}              (Eq. fmat)
 *   A_{mu lam i}= int phi_mu phi_lam / |r - r_i|            (Eq. 3c_grid)
 *   G_{mu i}    = w_i sum_lam A_{mu lam i} F_{lam i}        (Eq. gmat)
 *   Kt_{mu nu}  = sum_i G_{mu i} Phi_{nu i}                 (Eq. usym_k)
 *   K           = (Kt + Kt^T) / 2                           (Eq. sn_k)
 *   E_x         = -1/2 tr(P K)
 * with no screening, no batching and no approximation beyond the quadrature.
 *
 * The 3c-CP integrals are evaluated by the McMurchie-Davidson route of
 * Sec. II.B (Hermite expansion coefficients E, auxiliary integrals of
 * Eq. md1 seeded with the Boys function of Eq. boys), taken in the limit of a
 * unit point charge (the ket exponent to infinity, which turns the
 * 2 pi^{5/2}/(zeta_p zeta_c sqrt(zeta_p+zeta_c)) prefactor into 2 pi/zeta_p).
 * The GPU path uses the Obara-Saika recursions of App. A instead.
 *
 * The Boys function is summed from its positive series in extended precision
 * for x <= 40 + 6m and taken from its asymptotic form above (textbook method;
 * the paper gives none).
 *
 * Exact exchange from four-centre integrals (Eq. full_k, ERIs by the
 * McMurchie-Davidson formula generalised to four centres) is provided for
 * tiny systems, as the limit sn-K must converge to on grid refinement.
 *
 * Basis convention: shells of Cartesian Gaussians (l <= 2), components in
 * lexicographic order (x,y,z; xx,xy,xz,yy,yz,zz); the contraction
 * coefficients include the normalisation of the axis-aligned component and
 * every component is scaled to unit norm.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LMAX 2
#define ORC_L2 (2 * ORC_LMAX)       /* max l_a + l_b */
#define ORC_L4 (4 * ORC_LMAX)       /* max total for four-centre integrals */
/* above this argument the asymptotic form of F_m is exact to < 1e-20 relative */
#define ORC_BOYS_SWITCH(m) (40.0 + 6.0 * (m))

static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

static double dfact(int n) /* n!!, (-1)!! = 1 */
{
    double r = 1.0;
    while (n > 1) { r *= n; n -= 2; }
    return r;
}

/* Cartesian exponents of component c of a shell of angular momentum l. */
static void comp_of(int l, int c, int* lx, int* ly, int* lz)
{
    int k = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (k == c) { *lx = x; *ly = y; *lz = l - x - y; return; }
            ++k;
        }
}

/* factor that scales component (lx,ly,lz) of a shell to unit norm */
static double comp_norm(int l, int lx, int ly, int lz)
{
    return sqrt(dfact(2 * l - 1) / (dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1)));
}

int orc_nbf(int nshell, const int* l)
{
    int n = 0;
    for (int s = 0; s < nshell; ++s) n += ncart(l[s]);
    return n;
}

static void shell_offsets(int nshell, const int* l, int* off)
{
    off[0] = 0;
    for (int s = 0; s < nshell; ++s) off[s + 1] = off[s] + ncart(l[s]);
}

/* ------------------------------------------------------------------------ */
/* Boys function F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy        (Eq. boys)   */
/* ------------------------------------------------------------------------ */

double orc_boys(int m, double x)
{
    if (x > ORC_BOYS_SWITCH(m)) {
        /* F_m(x) = (2m-1)!! / 2^{m+1} * sqrt(pi / x^{2m+1}) */
        return dfact(2 * m - 1) / ldexp(1.0, m + 1) * sqrt(ORC_PI / pow(x, 2 * m + 1));
    }
    /* F_m(x) = e^{-x} sum_k (2x)^k / ((2m+1)(2m+3)...(2m+2k+1)), all terms positive */
    long double X = (long double)x;
    long double t = 1.0L / (2 * m + 1);
    long double s = t;
    for (int k = 1; k < 2000; ++k) {
        t *= 2.0L * X / (long double)(2 * m + 2 * k + 1);
        s += t;
        if (t < 1e-21L * s) break;
    }
    return (double)(expl(-X) * s);
}

/* F_0..F_mmax at one argument: the top order from the series (or the
 * asymptotic form), the lower ones by the downward recursion
 * F_m = (2x F_{m+1} + e^{-x}) / (2m+1), which follows from Eq. boys by parts. */
static void boys_all(int mmax, double x, double* F)
{
    if (x > ORC_BOYS_SWITCH(mmax)) {
        for (int m = 0; m <= mmax; ++m) F[m] = orc_boys(m, x);
        return;
    }
    long double X = (long double)x;
    long double t = 1.0L / (2 * mmax + 1);
    long double s = t;
    for (int k = 1; k < 2000; ++k) {
        t *= 2.0L * X / (long double)(2 * mmax + 2 * k + 1);
        s += t;
        if (t < 1e-21L * s) break;
    }
    const long double ex = expl(-X);
    long double fm = ex * s;
    F[mmax] = (double)fm;
    for (int m = mmax - 1; m >= 0; --m) {
        fm = (2.0L * X * fm + ex) / (long double)(2 * m + 1);
        F[m] = (double)fm;
    }
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson pieces                                                */
/* ------------------------------------------------------------------------ */

/* Hermite expansion coefficients E^{ij}_t of one Cartesian direction for the
 * product of x_A^i e^{-a x_A^2} and x_B^j e^{-b x_B^2}; XAB = A - B. */
static void md_E(int imax, int jmax, double a, double b, double XAB,
                 double E[ORC_LMAX + 1][ORC_LMAX + 1][ORC_L2 + 1])
{
    const double p = a + b, mu = a * b / p;
    const double XPA = -b / p * XAB, XPB = a / p * XAB, oo2p = 0.5 / p;
    memset(E, 0, sizeof(double) * (ORC_LMAX + 1) * (ORC_LMAX + 1) * (ORC_L2 + 1));
    E[0][0][0] = exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; ++i) {
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (i > 0) {
                    /* E^{i,j}_t from E^{i-1,j} */
                    v = XPA * E[i - 1][j][t];
                    if (t > 0) v += oo2p * E[i - 1][j][t - 1];
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                } else {
                    v = XPB * E[i][j - 1][t];
                    if (t > 0) v += oo2p * E[i][j - 1][t - 1];
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                }
                E[i][j][t] = v;
            }
        }
    }
}

/* Auxiliary Hermite integrals R^0_{tuv}, t+u+v <= L, by Eq. md1:
 *   R^n_{000} = (-2 alpha)^n F_n(alpha |PC|^2)
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PC R^{n+1}_{t,u,v}  (same for u, v). */
#define RDIM (ORC_L4 + 1)
static void md_R(int L, double alpha, const double PC[3], double R0[RDIM][RDIM][RDIM])
{
    static __thread double R[RDIM][RDIM][RDIM][RDIM];
    const double T = alpha * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
    double Fm[RDIM];
    boys_all(L, T, Fm);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) {
        R[n][0][0][0] = f * Fm[n];
        f *= -2.0 * alpha;
    }
    for (int tot = 1; tot <= L; ++tot) {
        for (int n = 0; n <= L - tot; ++n) {
            for (int t = tot; t >= 0; --t) {
                for (int u = tot - t; u >= 0; --u) {
                    int v = tot - t - u;
                    double val;
                    if (t > 0) {
                        val = PC[0] * R[n + 1][t - 1][u][v];
                        if (t > 1) val += (t - 1) * R[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        val = PC[1] * R[n + 1][t][u - 1][v];
                        if (u > 1) val += (u - 1) * R[n + 1][t][u - 2][v];
                    } else {
                        val = PC[2] * R[n + 1][t][u][v - 1];
                        if (v > 1) val += (v - 1) * R[n + 1][t][u][v - 2];
                    }
                    R[n][t][u][v] = val;
                }
            }
        }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) R0[t][u][v] = R[0][t][u][v];
}

/* C-independent data of one primitive pair */
typedef struct {
    double p, P[3], pref;                                   /* pref = c_a c_b */
    double E[3][ORC_LMAX + 1][ORC_LMAX + 1][ORC_L2 + 1];
} prim_pair;

typedef struct {
    int sa, sb, la, lb, npp;
    prim_pair* pp;
    int ea[6][3], eb[6][3];      /* Cartesian exponents of the components */
    double nra[6], nrb[6];       /* component norms */
} shell_pair;

static void make_shell_pair(shell_pair* sp, int sa, int sb, const double* center, const int* l,
                            const int* nprim, const int* prim_off, const double* exps, const double* coefs)
{
    sp->sa = sa; sp->sb = sb; sp->la = l[sa]; sp->lb = l[sb];
    sp->npp = nprim[sa] * nprim[sb];
    for (int c = 0; c < ncart(sp->la); ++c) {
        comp_of(sp->la, c, &sp->ea[c][0], &sp->ea[c][1], &sp->ea[c][2]);
        sp->nra[c] = comp_norm(sp->la, sp->ea[c][0], sp->ea[c][1], sp->ea[c][2]);
    }
    for (int c = 0; c < ncart(sp->lb); ++c) {
        comp_of(sp->lb, c, &sp->eb[c][0], &sp->eb[c][1], &sp->eb[c][2]);
        sp->nrb[c] = comp_norm(sp->lb, sp->eb[c][0], sp->eb[c][1], sp->eb[c][2]);
    }
    sp->pp = (prim_pair*)malloc(sizeof(prim_pair) * (size_t)sp->npp);
    const double* A = center + 3 * sa;
    const double* B = center + 3 * sb;
    int k = 0;
    for (int i = 0; i < nprim[sa]; ++i) {
        for (int j = 0; j < nprim[sb]; ++j, ++k) {
            double a = exps[prim_off[sa] + i], b = exps[prim_off[sb] + j];
            prim_pair* q = &sp->pp[k];
            q->p = a + b;
            for (int d = 0; d < 3; ++d) {
                q->P[d] = (a * A[d] + b * B[d]) / q->p;
                md_E(sp->la, sp->lb, a, b, A[d] - B[d], q->E[d]);
            }
            q->pref = coefs[prim_off[sa] + i] * coefs[prim_off[sb] + j];
        }
    }
}

/* Contracted 3c-CP block A_{ab}(C) = int phi_a phi_b / |r - C| for one shell pair,
 * written as out[ia * ncart(lb) + ib]. */
static void a3c_block(const shell_pair* sp, const double C[3], double* out)
{
    const int na = ncart(sp->la), nb = ncart(sp->lb), L = sp->la + sp->lb;
    double R0[RDIM][RDIM][RDIM];
    int ax[6], ay[6], az[6], bx[6], by[6], bz[6];
    const double* na_ = sp->nra;
    const double* nb_ = sp->nrb;
    for (int c = 0; c < na; ++c) { ax[c] = sp->ea[c][0]; ay[c] = sp->ea[c][1]; az[c] = sp->ea[c][2]; }
    for (int c = 0; c < nb; ++c) { bx[c] = sp->eb[c][0]; by[c] = sp->eb[c][1]; bz[c] = sp->eb[c][2]; }
    for (int k = 0; k < na * nb; ++k) out[k] = 0.0;
    for (int k = 0; k < sp->npp; ++k) {
        const prim_pair* q = &sp->pp[k];
        double PC[3] = {q->P[0] - C[0], q->P[1] - C[1], q->P[2] - C[2]};
        md_R(L, q->p, PC, R0);
        const double f = q->pref * 2.0 * ORC_PI / q->p;
        for (int ia = 0; ia < na; ++ia) {
            for (int ib = 0; ib < nb; ++ib) {
                double s = 0.0;
                for (int t = 0; t <= ax[ia] + bx[ib]; ++t)
                    for (int u = 0; u <= ay[ia] + by[ib]; ++u)
                        for (int v = 0; v <= az[ia] + bz[ib]; ++v)
                            s += q->E[0][ax[ia]][bx[ib]][t] * q->E[1][ay[ia]][by[ib]][u] *
                                 q->E[2][az[ia]][bz[ib]][v] * R0[t][u][v];
                out[ia * nb + ib] += f * s;
            }
        }
    }
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) out[ia * nb + ib] *= na_[ia] * nb_[ib];
}

/* ------------------------------------------------------------------------ */
/* collocation  Phi_{mu i} = phi_mu(r_i)                   (Eq. collocation) */
/* ------------------------------------------------------------------------ */

static void collocate_point(int nshell, const double* center, const int* l, const int* nprim,
                            const int* prim_off, const double* exps, const double* coefs,
                            const double r[3], double* phi)
{
    int mu = 0;
    for (int s = 0; s < nshell; ++s) {
        const double dx = r[0] - center[3 * s], dy = r[1] - center[3 * s + 1], dz = r[2] - center[3 * s + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        double radial = 0.0;
        for (int k = 0; k < nprim[s]; ++k) radial += coefs[prim_off[s] + k] * exp(-exps[prim_off[s] + k] * r2);
        for (int c = 0; c < ncart(l[s]); ++c) {
            int lx, ly, lz;
            comp_of(l[s], c, &lx, &ly, &lz);
            phi[mu++] = comp_norm(l[s], lx, ly, lz) * pow(dx, lx) * pow(dy, ly) * pow(dz, lz) * radial;
        }
    }
}

/* Phi is written as Phi[mu * npts + i]. */
void orc_collocate(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                   const double* exps, const double* coefs, long npts, const double* xyz, double* Phi)
{
    const int nbf = orc_nbf(nshell, l);
    double* phi = (double*)malloc(sizeof(double) * (size_t)nbf);
    for (long i = 0; i < npts; ++i) {
        collocate_point(nshell, center, l, nprim, prim_off, exps, coefs, xyz + 3 * i, phi);
        for (int mu = 0; mu < nbf; ++mu) Phi[(size_t)mu * npts + i] = phi[mu];
    }
    free(phi);
}

/* ------------------------------------------------------------------------ */
/* overlap and one-point 3c-CP matrices (pins)                              */
/* ------------------------------------------------------------------------ */

/* S_{ab} = (pi/p)^{3/2} E^{ab}_0(x) E^{ab}_0(y) E^{ab}_0(z), contracted */
void orc_overlap(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                 const double* exps, const double* coefs, double* S)
{
    const int nbf = orc_nbf(nshell, l);
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    for (int sa = 0; sa < nshell; ++sa) {
        for (int sb = 0; sb < nshell; ++sb) {
            shell_pair sp;
            make_shell_pair(&sp, sa, sb, center, l, nprim, prim_off, exps, coefs);
            for (int ia = 0; ia < ncart(l[sa]); ++ia) {
                int ax, ay, az;
                comp_of(l[sa], ia, &ax, &ay, &az);
                for (int ib = 0; ib < ncart(l[sb]); ++ib) {
                    int bx, by, bz;
                    comp_of(l[sb], ib, &bx, &by, &bz);
                    double s = 0.0;
                    for (int k = 0; k < sp.npp; ++k) {
                        const prim_pair* q = &sp.pp[k];
                        s += q->pref * pow(ORC_PI / q->p, 1.5) * q->E[0][ax][bx][0] * q->E[1][ay][by][0] *
                             q->E[2][az][bz][0];
                    }
                    S[(size_t)(off[sa] + ia) * nbf + off[sb] + ib] =
                        s * comp_norm(l[sa], ax, ay, az) * comp_norm(l[sb], bx, by, bz);
                }
            }
            free(sp.pp);
        }
    }
    free(off);
}

/* Full A(C) matrix (nbf x nbf, row-major) at one point C. */
void orc_a3c(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
             const double* exps, const double* coefs, const double* C, double* A)
{
    const int nbf = orc_nbf(nshell, l);
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    double blk[36];
    for (int sa = 0; sa < nshell; ++sa) {
        for (int sb = 0; sb < nshell; ++sb) {
            shell_pair sp;
            make_shell_pair(&sp, sa, sb, center, l, nprim, prim_off, exps, coefs);
            a3c_block(&sp, C, blk);
            for (int ia = 0; ia < ncart(l[sa]); ++ia)
                for (int ib = 0; ib < ncart(l[sb]); ++ib)
                    A[(size_t)(off[sa] + ia) * nbf + off[sb] + ib] = blk[ia * ncart(l[sb]) + ib];
            free(sp.pp);
        }
    }
    free(off);
}

/* ------------------------------------------------------------------------ */
/* sn-K (Eqs. fmat, gmat, usym_k, sn_k)                                     */
/* ------------------------------------------------------------------------ */

static void kahan_add(double* sum, double* comp, double x)
{
    double y = x - *comp;
    double t = *sum + y;
    *comp = (t - *sum) - y;
    *sum = t;
}

/*
 * K (nbf x nbf, row-major, overwritten) and two evaluations of E_x:
 *   ex[0] = -1/2 tr(P K)   and   ex[1] = -1/2 sum_{mu,i} F_{mu i} G_{mu i}.
 * Points are split into fixed contiguous chunks; each chunk accumulates its
 * partial Kt in point order and the partials are added pairwise, so the result
 * does not depend on the number of threads.  Returns 0 on success.
 */
int orc_snk(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
            const double* exps, const double* coefs, long npts, const double* xyz, const double* w,
            const double* P, double* K, double* ex, int nthreads)
{
    const int nbf = orc_nbf(nshell, l);
    const size_t nb2 = (size_t)nbf * nbf;
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);

    /* unique shell pairs a >= b with their C-independent primitive data */
    const int npair = nshell * (nshell + 1) / 2;
    shell_pair* sps = (shell_pair*)malloc(sizeof(shell_pair) * (size_t)npair);
    {
        int k = 0;
        for (int sa = 0; sa < nshell; ++sa)
            for (int sb = 0; sb <= sa; ++sb)
                make_shell_pair(&sps[k++], sa, sb, center, l, nprim, prim_off, exps, coefs);
    }

    int nchunk = 64;
    if (npts < nchunk) nchunk = npts > 0 ? (int)npts : 1;
    double* part = (double*)calloc((size_t)nchunk * nb2, sizeof(double));
    double* fg = (double*)calloc((size_t)nchunk * 2, sizeof(double));
    if (!part || !fg) return 1;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double* A = (double*)malloc(sizeof(double) * nb2);
        double* phi = (double*)malloc(sizeof(double) * (size_t)nbf);
        double* f = (double*)malloc(sizeof(double) * (size_t)nbf);
        double* g = (double*)malloc(sizeof(double) * (size_t)nbf);
        double blk[36];
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < nchunk; ++c) {
            const long i0 = npts * c / nchunk, i1 = npts * (c + 1) / nchunk;
            double* Kt = part + (size_t)c * nb2;
            double s_fg = 0.0, c_fg = 0.0;
            for (long i = i0; i < i1; ++i) {
                const double* r = xyz + 3 * i;
                collocate_point(nshell, center, l, nprim, prim_off, exps, coefs, r, phi);
                /* F_{lam i} = sum_nu P_{lam nu} Phi_{nu i} */
                for (int lam = 0; lam < nbf; ++lam) {
                    double s = 0.0;
                    for (int nu = 0; nu < nbf; ++nu) s += P[(size_t)lam * nbf + nu] * phi[nu];
                    f[lam] = s;
                }
                /* A(r_i), both triangles (A_{mu lam} = A_{lam mu}) */
                for (int k = 0; k < npair; ++k) {
                    const shell_pair* sp = &sps[k];
                    const int na = ncart(sp->la), nbb = ncart(sp->lb);
                    a3c_block(sp, r, blk);
                    for (int ia = 0; ia < na; ++ia)
                        for (int ib = 0; ib < nbb; ++ib) {
                            const double v = blk[ia * nbb + ib];
                            A[(size_t)(off[sp->sa] + ia) * nbf + off[sp->sb] + ib] = v;
                            A[(size_t)(off[sp->sb] + ib) * nbf + off[sp->sa] + ia] = v;
                        }
                }
                /* G_{mu i} = w_i sum_lam A_{mu lam} F_{lam i} */
                for (int mu = 0; mu < nbf; ++mu) {
                    double s = 0.0;
                    for (int lam = 0; lam < nbf; ++lam) s += A[(size_t)mu * nbf + lam] * f[lam];
                    g[mu] = w[i] * s;
                }
                /* Kt_{mu nu} += G_{mu i} Phi_{nu i} */
                for (int mu = 0; mu < nbf; ++mu) {
                    const double gm = g[mu];
                    double* row = Kt + (size_t)mu * nbf;
                    for (int nu = 0; nu < nbf; ++nu) row[nu] += gm * phi[nu];
                }
                for (int mu = 0; mu < nbf; ++mu) kahan_add(&s_fg, &c_fg, f[mu] * g[mu]);
            }
            fg[2 * c] = s_fg;
            fg[2 * c + 1] = c_fg;
        }
        free(A); free(phi); free(f); free(g);
    }

    /* pairwise sum of the chunk partials */
    for (int stride = 1; stride < nchunk; stride *= 2)
        for (int c = 0; c + stride < nchunk; c += 2 * stride) {
            double* dst = part + (size_t)c * nb2;
            const double* src = part + (size_t)(c + stride) * nb2;
            for (size_t k = 0; k < nb2; ++k) dst[k] += src[k];
        }
    const double* Kt = part;
    for (int mu = 0; mu < nbf; ++mu)
        for (int nu = 0; nu < nbf; ++nu)
            K[(size_t)mu * nbf + nu] = 0.5 * (Kt[(size_t)mu * nbf + nu] + Kt[(size_t)nu * nbf + mu]);

    double s = 0.0, cp = 0.0;
    for (int mu = 0; mu < nbf; ++mu)
        for (int nu = 0; nu < nbf; ++nu) kahan_add(&s, &cp, P[(size_t)mu * nbf + nu] * K[(size_t)nu * nbf + mu]);
    ex[0] = -0.5 * s;
    s = 0.0; cp = 0.0;
    for (int c = 0; c < nchunk; ++c) { kahan_add(&s, &cp, fg[2 * c]); kahan_add(&s, &cp, -fg[2 * c + 1]); }
    ex[1] = -0.5 * s;

    for (int k = 0; k < npair; ++k) free(sps[k].pp);
    free(sps); free(part); free(fg); free(off);
    return 0;
}

/*
 * Selected rows of the unsymmetrised sn-K matrix (Eqs. fmat, 3c_grid, gmat, usym_k):
 *   Kt_rows[r][nu] = sum_i G_{mu_r i} Phi_{nu i},   G_{mu i} = w_i sum_lam A_{mu lam}(r_i) F_{lam i},
 * for mu_r = rows[r], r < nrows (nrows x nbf, row-major, overwritten).  The same definition as
 * orc_snk, restricted to the rows asked for, so that matrices too large for the full product
 * can be sampled: K_{mu nu} = (Kt_{mu nu} + Kt_{nu mu}) / 2 for mu, nu both among the rows.
 * Points are split into fixed chunks summed pairwise (thread-count independent).
 */
int orc_snk_rows(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                 const double* exps, const double* coefs, long npts, const double* xyz, const double* w,
                 const double* P, const int* rows, int nrows, double* Kt_rows, int nthreads)
{
    const int nbf = orc_nbf(nshell, l);
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    int* shell_of = (int*)malloc(sizeof(int) * (size_t)nbf);
    for (int sh = 0; sh < nshell; ++sh)
        for (int k = off[sh]; k < off[sh + 1]; ++k) shell_of[k] = sh;
    /* the shell pairs (row shell, any shell) */
    shell_pair* sps = (shell_pair*)malloc(sizeof(shell_pair) * (size_t)nrows * nshell);
    for (int r = 0; r < nrows; ++r)
        for (int sb = 0; sb < nshell; ++sb)
            make_shell_pair(&sps[(size_t)r * nshell + sb], shell_of[rows[r]], sb, center, l, nprim, prim_off, exps,
                            coefs);
    const size_t nout = (size_t)nrows * nbf;
    int nchunk = 64;
    if (npts < nchunk) nchunk = npts > 0 ? (int)npts : 1;
    double* part = (double*)calloc((size_t)nchunk * nout, sizeof(double));
    if (!part) return 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double* phi = (double*)malloc(sizeof(double) * (size_t)nbf);
        double* f = (double*)malloc(sizeof(double) * (size_t)nbf);
        double blk[36];
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < nchunk; ++c) {
            const long i0 = npts * c / nchunk, i1 = npts * (c + 1) / nchunk;
            double* Kt = part + (size_t)c * nout;
            for (long i = i0; i < i1; ++i) {
                const double* rp = xyz + 3 * i;
                collocate_point(nshell, center, l, nprim, prim_off, exps, coefs, rp, phi);
                for (int lam = 0; lam < nbf; ++lam) {
                    double s = 0.0;
                    for (int nu = 0; nu < nbf; ++nu) s += P[(size_t)lam * nbf + nu] * phi[nu];
                    f[lam] = s;
                }
                for (int r = 0; r < nrows; ++r) {
                    const int mu = rows[r], sa = shell_of[mu], ia = mu - off[sa];
                    double s = 0.0;
                    for (int sb = 0; sb < nshell; ++sb) {
                        const shell_pair* sp = &sps[(size_t)r * nshell + sb];
                        const int nbb = ncart(sp->lb);
                        a3c_block(sp, rp, blk);
                        for (int ib = 0; ib < nbb; ++ib) s += blk[ia * nbb + ib] * f[off[sb] + ib];
                    }
                    const double g = w[i] * s;
                    double* row = Kt + (size_t)r * nbf;
                    for (int nu = 0; nu < nbf; ++nu) row[nu] += g * phi[nu];
                }
            }
        }
        free(phi); free(f);
    }
    for (int stride = 1; stride < nchunk; stride *= 2)
        for (int c = 0; c + stride < nchunk; c += 2 * stride) {
            double* dst = part + (size_t)c * nout;
            const double* src = part + (size_t)(c + stride) * nout;
            for (size_t k = 0; k < nout; ++k) dst[k] += src[k];
        }
    for (size_t k = 0; k < nout; ++k) Kt_rows[k] = part[k];
    for (size_t k = 0; k < (size_t)nrows * nshell; ++k) free(sps[k].pp);
    free(sps); free(part); free(off); free(shell_of);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exact exchange from four-centre ERIs (Eq. full_k)                        */
/* ------------------------------------------------------------------------ */

/* Contracted ERI block (ab|cd) over shells, out[((ia*nb+ib)*nc+ic)*nd+id]:
 *   (ab|cd) = 2 pi^{5/2}/(p q sqrt(p+q)) sum_{tuv} E^{ab}_{tuv}
 *             sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi}(pq/(p+q), P-Q) */
static void eri_block(const shell_pair* ab, const shell_pair* cd, double* out)
{
    const int na = ncart(ab->la), nb = ncart(ab->lb), nc = ncart(cd->la), nd = ncart(cd->lb);
    const int L = ab->la + ab->lb + cd->la + cd->lb;
    int e[4][6][3];
    double nrm[4][6];
    const int ls[4] = {ab->la, ab->lb, cd->la, cd->lb};
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < ncart(ls[s]); ++c) {
            comp_of(ls[s], c, &e[s][c][0], &e[s][c][1], &e[s][c][2]);
            nrm[s][c] = comp_norm(ls[s], e[s][c][0], e[s][c][1], e[s][c][2]);
        }
    const int n = na * nb * nc * nd;
    for (int k = 0; k < n; ++k) out[k] = 0.0;
    double R0[RDIM][RDIM][RDIM];
    for (int k1 = 0; k1 < ab->npp; ++k1) {
        const prim_pair* q1 = &ab->pp[k1];
        for (int k2 = 0; k2 < cd->npp; ++k2) {
            const prim_pair* q2 = &cd->pp[k2];
            const double p = q1->p, q = q2->p, alpha = p * q / (p + q);
            const double PQ[3] = {q1->P[0] - q2->P[0], q1->P[1] - q2->P[1], q1->P[2] - q2->P[2]};
            md_R(L, alpha, PQ, R0);
            const double f = q1->pref * q2->pref * 2.0 * pow(ORC_PI, 2.5) / (p * q * sqrt(p + q));
            int k = 0;
            for (int ia = 0; ia < na; ++ia)
                for (int ib = 0; ib < nb; ++ib)
                    for (int ic = 0; ic < nc; ++ic)
                        for (int id = 0; id < nd; ++id, ++k) {
                            const int *A = e[0][ia], *B = e[1][ib], *Cc = e[2][ic], *D = e[3][id];
                            double s = 0.0;
                            for (int t = 0; t <= A[0] + B[0]; ++t)
                                for (int u = 0; u <= A[1] + B[1]; ++u)
                                    for (int v = 0; v <= A[2] + B[2]; ++v) {
                                        const double eab = q1->E[0][A[0]][B[0]][t] * q1->E[1][A[1]][B[1]][u] *
                                                           q1->E[2][A[2]][B[2]][v];
                                        double inner = 0.0;
                                        for (int ta = 0; ta <= Cc[0] + D[0]; ++ta)
                                            for (int nu = 0; nu <= Cc[1] + D[1]; ++nu)
                                                for (int ph = 0; ph <= Cc[2] + D[2]; ++ph) {
                                                    const double sg = ((ta + nu + ph) & 1) ? -1.0 : 1.0;
                                                    inner += sg * q2->E[0][Cc[0]][D[0]][ta] *
                                                             q2->E[1][Cc[1]][D[1]][nu] *
                                                             q2->E[2][Cc[2]][D[2]][ph] * R0[t + ta][u + nu][v + ph];
                                                }
                                        s += eab * inner;
                                    }
                            out[k] += f * s;
                        }
        }
    }
    int k = 0;
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib)
            for (int ic = 0; ic < nc; ++ic)
                for (int id = 0; id < nd; ++id, ++k) out[k] *= nrm[0][ia] * nrm[1][ib] * nrm[2][ic] * nrm[3][id];
}

/* One contracted ERI block over shells (sa sb | sc sd). */
void orc_eri_shells(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                    const double* exps, const double* coefs, int sa, int sb, int sc, int sd, double* out)
{
    (void)nshell;
    shell_pair ab, cd;
    make_shell_pair(&ab, sa, sb, center, l, nprim, prim_off, exps, coefs);
    make_shell_pair(&cd, sc, sd, center, l, nprim, prim_off, exps, coefs);
    eri_block(&ab, &cd, out);
    free(ab.pp);
    free(cd.pp);
}

/* K_{mu nu} = sum_{lam kap} (mu lam | nu kap) P_{lam kap}, all quartets, no screening. */
int orc_eri_k(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
              const double* exps, const double* coefs, const double* P, double* K, int nthreads)
{
    const int nbf = orc_nbf(nshell, l);
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    shell_pair* sps = (shell_pair*)malloc(sizeof(shell_pair) * (size_t)nshell * nshell);
    for (int a = 0; a < nshell; ++a)
        for (int b = 0; b < nshell; ++b)
            make_shell_pair(&sps[a * nshell + b], a, b, center, l, nprim, prim_off, exps, coefs);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* each (a, c) shell block of K is owned by one iteration */
#pragma omp parallel
    {
        double* blk = (double*)malloc(sizeof(double) * 1296);
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int a = 0; a < nshell; ++a) {
            for (int c = 0; c < nshell; ++c) {
                const int na = ncart(l[a]), nc = ncart(l[c]);
                double acc[36];
                for (int k = 0; k < 36; ++k) acc[k] = 0.0;
                for (int b = 0; b < nshell; ++b) {
                    for (int d = 0; d < nshell; ++d) {
                        const int nb = ncart(l[b]), nd = ncart(l[d]);
                        eri_block(&sps[a * nshell + b], &sps[c * nshell + d], blk);
                        for (int ia = 0; ia < na; ++ia)
                            for (int ib = 0; ib < nb; ++ib)
                                for (int ic = 0; ic < nc; ++ic)
                                    for (int id = 0; id < nd; ++id)
                                        acc[ia * nc + ic] += blk[((ia * nb + ib) * nc + ic) * nd + id] *
                                                             P[(size_t)(off[b] + ib) * nbf + off[d] + id];
                    }
                }
                for (int ia = 0; ia < na; ++ia)
                    for (int ic = 0; ic < nc; ++ic) K[(size_t)(off[a] + ia) * nbf + off[c] + ic] = acc[ia * nc + ic];
            }
        }
        free(blk);
    }
    for (int k = 0; k < nshell * nshell; ++k) free(sps[k].pp);
    free(sps);
    free(off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* density-fitting tensors (Sec. II.B, Eqs. V_df, P_df, J_df)               */
/* ------------------------------------------------------------------------ */

/*
 * Three- and two-centre Coulomb integrals of the density-fitting approximation over one
 * combined shell list: shells [0, norb) are the orbital basis, shells [norb, norb + naux)
 * the auxiliary basis, and shell norb + naux must be an s function of exponent 0 and
 * coefficient 1 (the constant function 1), so that by the definitions
 *   (mu nu | K) = (mu nu | K 1)   and   (K | L) = (K 1 | L 1)
 * both come from the four-centre routine above.  Outputs (row-major, overwritten):
 *   T[(mu * nbf + nu) * nauxf + K] = (mu nu | K)     nbf x nbf x nauxf
 *   V[K * nauxf + L]                = (K | L)          nauxf x nauxf
 * Returns 0 on success, -1 if the last shell is not the constant function.
 */
int orc_df_tensors(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                   const double* exps, const double* coefs, int norb, int naux, double* T, double* V,
                   int nthreads)
{
    const int one = norb + naux;
    if (one != nshell - 1 || l[one] != 0 || nprim[one] != 1 || exps[prim_off[one]] != 0.0 ||
        coefs[prim_off[one]] != 1.0)
        return -1;
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    const int nbf = off[norb], nauxf = off[norb + naux] - off[norb];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* the auxiliary functions paired with the constant */
    shell_pair* kp = (shell_pair*)malloc(sizeof(shell_pair) * (size_t)(naux > 0 ? naux : 1));
    for (int k = 0; k < naux; ++k)
        make_shell_pair(&kp[k], norb + k, one, center, l, nprim, prim_off, exps, coefs);
    const int npair = norb * (norb + 1) / 2;
#pragma omp parallel
    {
        double* blk = (double*)malloc(sizeof(double) * 1296);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npair; ++p) {
            int a = 0;
            while ((a + 1) * (a + 2) / 2 <= p) ++a;
            const int b = p - a * (a + 1) / 2;
            shell_pair ab;
            make_shell_pair(&ab, a, b, center, l, nprim, prim_off, exps, coefs);
            const int na = ncart(l[a]), nb = ncart(l[b]);
            for (int k = 0; k < naux; ++k) {
                const int nk = ncart(l[norb + k]), k0 = off[norb + k] - nbf;
                eri_block(&ab, &kp[k], blk);
                for (int ia = 0; ia < na; ++ia)
                    for (int ib = 0; ib < nb; ++ib)
                        for (int ik = 0; ik < nk; ++ik) {
                            const double v = blk[(ia * nb + ib) * nk + ik];
                            T[((size_t)(off[a] + ia) * nbf + off[b] + ib) * nauxf + k0 + ik] = v;
                            T[((size_t)(off[b] + ib) * nbf + off[a] + ia) * nauxf + k0 + ik] = v;
                        }
            }
            free(ab.pp);
        }
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < naux; ++k) {
            const int nk = ncart(l[norb + k]), k0 = off[norb + k] - nbf;
            for (int m = 0; m < naux; ++m) {
                const int nm = ncart(l[norb + m]), m0 = off[norb + m] - nbf;
                eri_block(&kp[k], &kp[m], blk);
                for (int ik = 0; ik < nk; ++ik)
                    for (int im = 0; im < nm; ++im) V[(size_t)(k0 + ik) * nauxf + m0 + im] = blk[ik * nm + im];
            }
        }
        free(blk);
    }
    for (int k = 0; k < naux; ++k) free(kp[k].pp);
    free(kp);
    free(off);
    return 0;
}

/* J_{mu nu} = sum_{lam kap} (mu nu | lam kap) P_{lam kap}, all quartets, no screening. */
int orc_eri_j(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
              const double* exps, const double* coefs, const double* P, double* J, int nthreads)
{
    const int nbf = orc_nbf(nshell, l);
    int* off = (int*)malloc(sizeof(int) * (size_t)(nshell + 1));
    shell_offsets(nshell, l, off);
    shell_pair* sps = (shell_pair*)malloc(sizeof(shell_pair) * (size_t)nshell * nshell);
    for (int a = 0; a < nshell; ++a)
        for (int b = 0; b < nshell; ++b)
            make_shell_pair(&sps[a * nshell + b], a, b, center, l, nprim, prim_off, exps, coefs);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* each (a, b) shell block of J is owned by one iteration */
#pragma omp parallel
    {
        double* blk = (double*)malloc(sizeof(double) * 1296);
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int a = 0; a < nshell; ++a) {
            for (int b = 0; b < nshell; ++b) {
                const int na = ncart(l[a]), nb = ncart(l[b]);
                double acc[36];
                for (int k = 0; k < 36; ++k) acc[k] = 0.0;
                for (int c = 0; c < nshell; ++c) {
                    for (int d = 0; d < nshell; ++d) {
                        const int nc = ncart(l[c]), nd = ncart(l[d]);
                        eri_block(&sps[a * nshell + b], &sps[c * nshell + d], blk);
                        for (int ia = 0; ia < na; ++ia)
                            for (int ib = 0; ib < nb; ++ib)
                                for (int ic = 0; ic < nc; ++ic)
                                    for (int id = 0; id < nd; ++id)
                                        acc[ia * nb + ib] += blk[((ia * nb + ib) * nc + ic) * nd + id] *
                                                             P[(size_t)(off[c] + ic) * nbf + off[d] + id];
                    }
                }
                for (int ia = 0; ia < na; ++ia)
                    for (int ib = 0; ib < nb; ++ib) J[(size_t)(off[a] + ia) * nbf + off[b] + ib] = acc[ia * nb + ib];
            }
        }
        free(blk);
    }
    for (int k = 0; k < nshell * nshell; ++k) free(sps[k].pp);
    free(sps);
    free(off);
    return 0;
}
