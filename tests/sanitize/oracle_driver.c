/* Drives every entry point of the CPU oracle on a small s/p/d system so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check its memory accesses and
 * arithmetic.  Exit status 0 and "oracle driver ok" on success; the sanitizers abort on
 * the first error they find. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_nbf(int nshell, const int* l);
double orc_boys(int m, double x);
void orc_collocate(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                   const double* exps, const double* coefs, long npts, const double* xyz, double* Phi);
void orc_overlap(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                 const double* exps, const double* coefs, double* S);
void orc_a3c(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
             const double* exps, const double* coefs, const double* C, double* A);
int orc_snk(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
            const double* exps, const double* coefs, long npts, const double* xyz, const double* w,
            const double* P, double* K, double* ex, int nthreads);
int orc_snk_rows(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                 const double* exps, const double* coefs, long npts, const double* xyz, const double* w,
                 const double* P, const int* rows, int nrows, double* Kt_rows, int nthreads);
void orc_eri_shells(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
                    const double* exps, const double* coefs, int sa, int sb, int sc, int sd, double* out);
int orc_eri_k(int nshell, const double* center, const int* l, const int* nprim, const int* prim_off,
              const double* exps, const double* coefs, const double* P, double* K, int nthreads);

static int finite_all(const double* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            fprintf(stderr, "oracle driver: %s\n", what);   \
            return 1;                                       \
        }                                                   \
    } while (0)

int main(void)
{
    /* two centres: s (2 primitives), p, d on the first; s and p on the second */
    enum { NS = 5 };
    const double center[3 * NS] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1.1, 0.4, -0.3, 1.1, 0.4, -0.3};
    const int l[NS] = {0, 1, 2, 0, 1};
    const int nprim[NS] = {2, 1, 2, 1, 3};
    const int prim_off[NS] = {0, 2, 3, 5, 6};
    const double exps[9] = {3.0, 0.6, 1.2, 2.0, 0.5, 0.9, 30.0, 2.5, 0.35};
    const double coefs[9] = {0.7, 0.5, 1.0, 0.6, 0.6, 1.0, 0.2, 0.5, 0.6};
    const int nbf = orc_nbf(NS, l);
    CHECK(nbf == 1 + 3 + 6 + 1 + 3, "function count");

    for (int m = 0; m <= 8; ++m)
        for (double x = 0.0; x < 120.0; x = x * 1.7 + 0.01) CHECK(isfinite(orc_boys(m, x)), "Boys value");

    enum { NP = 37 };
    double xyz[3 * NP], w[NP];
    for (int i = 0; i < NP; ++i) {
        xyz[3 * i] = 0.31 * (i % 7) - 0.9;
        xyz[3 * i + 1] = 0.23 * (i % 5) - 0.4;
        xyz[3 * i + 2] = 0.17 * i - 2.0;
        w[i] = 0.05 + 0.01 * (i % 3);
    }
    double* Phi = malloc(sizeof(double) * (size_t)nbf * NP);
    double* S = malloc(sizeof(double) * (size_t)nbf * nbf);
    double* A = malloc(sizeof(double) * (size_t)nbf * nbf);
    double* P = malloc(sizeof(double) * (size_t)nbf * nbf);
    double* K = malloc(sizeof(double) * (size_t)nbf * nbf);
    double* K1 = malloc(sizeof(double) * (size_t)nbf * nbf);
    double* Kr = malloc(sizeof(double) * (size_t)3 * nbf);
    double* eri = malloc(sizeof(double) * 6 * 6 * 6 * 6);
    double ex[2] = {0.0, 0.0};
    for (int a = 0; a < nbf; ++a)
        for (int b = 0; b <= a; ++b) P[a * nbf + b] = P[b * nbf + a] = 0.3 / (1.0 + a + b) + (a == b ? 0.5 : 0.0);

    orc_collocate(NS, center, l, nprim, prim_off, exps, coefs, NP, xyz, Phi);
    CHECK(finite_all(Phi, (size_t)nbf * NP), "collocation");
    orc_overlap(NS, center, l, nprim, prim_off, exps, coefs, S);
    CHECK(finite_all(S, (size_t)nbf * nbf), "overlap");
    orc_a3c(NS, center, l, nprim, prim_off, exps, coefs, xyz + 3 * 5, A);
    CHECK(finite_all(A, (size_t)nbf * nbf), "three-centre integrals");
    CHECK(orc_snk(NS, center, l, nprim, prim_off, exps, coefs, NP, xyz, w, P, K, ex, 1) == 0, "sn-K");
    CHECK(finite_all(K, (size_t)nbf * nbf) && isfinite(ex[0]) && isfinite(ex[1]), "sn-K values");
    CHECK(orc_snk(NS, center, l, nprim, prim_off, exps, coefs, NP, xyz, w, P, K1, ex, 3) == 0, "sn-K threads");
    for (int k = 0; k < nbf * nbf; ++k) CHECK(K[k] == K1[k], "sn-K thread independence");
    const int rows[3] = {0, 5, nbf - 1};
    CHECK(orc_snk_rows(NS, center, l, nprim, prim_off, exps, coefs, NP, xyz, w, P, rows, 3, Kr, 2) == 0, "rows");
    CHECK(finite_all(Kr, (size_t)3 * nbf), "row values");
    orc_eri_shells(NS, center, l, nprim, prim_off, exps, coefs, 2, 1, 4, 0, eri);
    CHECK(finite_all(eri, 6 * 3 * 3 * 1), "ERI block");
    CHECK(orc_eri_k(NS, center, l, nprim, prim_off, exps, coefs, P, K1, 2) == 0, "four-centre K");
    CHECK(finite_all(K1, (size_t)nbf * nbf), "four-centre K values");
    /* an empty grid gives K = 0 */
    CHECK(orc_snk(NS, center, l, nprim, prim_off, exps, coefs, 0, xyz, w, P, K, ex, 1) == 0, "empty grid");
    for (int k = 0; k < nbf * nbf; ++k) CHECK(K[k] == 0.0, "empty grid K");

    free(Phi);
    free(S);
    free(A);
    free(P);
    free(K);
    free(K1);
    free(Kr);
    free(eri);
    printf("oracle driver ok\n");
    return 0;
}
