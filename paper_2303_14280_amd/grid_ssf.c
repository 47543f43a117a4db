/* Molecular-grid partition weights of Stratmann, Scuseria and Frisch (the weight scheme the
 * paper uses with its Mura-Knowles x Lebedev atomic grids, Sec. II.C), evaluated exactly.
 *
 * Part of the seeded input generator: it produces grid weights (input data) and nothing of
 * the exchange build.  Built with gcc by synth.py on first use.
 *
 * The cell function of the scheme is
 *     s(mu) = 1                                  for mu <= -a
 *           = 0                                  for mu >=  a
 *           = (1 - g(mu / a)) / 2,  g(x) = (35x - 35x^3 + 21x^5 - 5x^7) / 16   otherwise,
 * with a = 0.64 and mu_BC(r) = (|r - B| - |r - C|) / |B - C|.  The cell weight of atom B is
 * P_B(r) = prod_{C != B} s(mu_BC(r)) and a point r of atom p's grid gets the factor
 * P_p(r) / sum_B P_B(r).
 *
 * Because s is exactly 1 below -a and exactly 0 above a, the sums and products can be cut
 * without approximation:
 *  - if |r - p| <= (1 - a)/2 * (distance from p to its nearest atom) every mu_pC <= -a, so
 *    P_p = 1 and every other P_B contains s(mu_Bp) = 0: the factor is exactly 1;
 *  - with A the atom nearest to r, any B with |r - B| >= kappa |r - A|, kappa = (1+a)/(1-a),
 *    has mu_BA >= a (|A - B| <= |r - A| + |r - B|), hence P_B = 0;
 *  - in P_B a factor s(mu_BC) with |r - C| >= kappa |r - B| has mu_BC <= -a, hence is 1;
 *  - a single factor s(mu_BC) = 0 (mu_BC >= a) makes P_B = 0.
 * Every remaining factor is evaluated, so the result is the scheme's weight to rounding.
 */
#include <math.h>
#include <stdlib.h>

static const double kA = 0.64;

static double ssf_s(double mu)
{
    if (mu <= -kA) return 1.0;
    if (mu >= kA) return 0.0;
    const double x = mu / kA, x2 = x * x;
    const double g = x * (35.0 + x2 * (-35.0 + x2 * (21.0 - 5.0 * x2))) / 16.0;
    const double v = 0.5 * (1.0 - g);   /* |g| may round past 1 next to |x| = 1 */
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

/* natom atoms (xyz, bohr); npts points (xyz) with their parent atom; out[i] = partition factor.
 * Returns 0, or -1 when memory runs out. */
int ssf_weights(int natom, const double* atoms, long npts, const double* pts, const int* parent, double* out)
{
    const double kappa = (1.0 + kA) / (1.0 - kA);
    double* inv_r = (double*)malloc(sizeof(double) * (size_t)natom * (size_t)natom);
    double* rnn = (double*)malloc(sizeof(double) * (size_t)natom);
    if (!inv_r || !rnn) {
        free(inv_r);
        free(rnn);
        return -1;
    }
    for (int b = 0; b < natom; ++b) {
        rnn[b] = INFINITY;
        for (int c = 0; c < natom; ++c) {
            const double dx = atoms[3 * b] - atoms[3 * c], dy = atoms[3 * b + 1] - atoms[3 * c + 1],
                         dz = atoms[3 * b + 2] - atoms[3 * c + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            inv_r[(size_t)b * natom + c] = c == b ? 0.0 : 1.0 / r;
            if (c != b && r < rnn[b]) rnn[b] = r;
        }
    }
    int fail = 0;
#pragma omp parallel
    {
        double* d = (double*)malloc(sizeof(double) * (size_t)natom);
        int* cand = (int*)malloc(sizeof(int) * (size_t)natom);
        int* near = (int*)malloc(sizeof(int) * (size_t)natom);
        if (!d || !cand || !near) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1024)
        for (long i = 0; i < npts; ++i) {
            if (!d || !cand || !near) continue;
            const int p = parent[i];
            const double* r = pts + 3 * i;
            const double dxp = r[0] - atoms[3 * p], dyp = r[1] - atoms[3 * p + 1], dzp = r[2] - atoms[3 * p + 2];
            const double dp = sqrt(dxp * dxp + dyp * dyp + dzp * dzp);
            if (dp <= 0.5 * (1.0 - kA) * rnn[p]) {
                out[i] = 1.0;
                continue;
            }
            double dmin = INFINITY;
            int amin = 0;
            for (int c = 0; c < natom; ++c) {
                const double dx = r[0] - atoms[3 * c], dy = r[1] - atoms[3 * c + 1], dz = r[2] - atoms[3 * c + 2];
                d[c] = sqrt(dx * dx + dy * dy + dz * dz);
                if (d[c] < dmin) {
                    dmin = d[c];
                    amin = c;
                }
            }
            /* the parent's weight is zero when the nearest atom alone forces it */
            if (d[p] >= kappa * dmin || (p != amin && (d[p] - dmin) * inv_r[(size_t)p * natom + amin] >= kA)) {
                out[i] = 0.0;
                continue;
            }
            /* atoms that can carry a non-zero P_B, nearest first */
            int nc = 0, nn = 0;
            const double lim_c = kappa * dmin;
            for (int c = 0; c < natom; ++c)
                if (d[c] < lim_c) {
                    int k = nc++;
                    while (k > 0 && d[cand[k - 1]] > d[c]) {
                        cand[k] = cand[k - 1];
                        --k;
                    }
                    cand[k] = c;
                }
            /* drop those that another such atom zeroes (s(mu_BC) = 0 for mu_BC >= a) */
            int ns = 0;
            double dbmax = 0.0;
            for (int q = 0; q < nc; ++q) {
                const int b = cand[q];
                const double* ir = inv_r + (size_t)b * natom;
                int alive = 1;
                for (int k = 0; k < nc && alive; ++k) {
                    const int c = cand[k];
                    if (c != b && (d[b] - d[c]) * ir[c] >= kA) alive = 0;
                }
                if (alive) {
                    cand[ns++] = b;
                    if (d[b] > dbmax) dbmax = d[b];
                }
            }
            /* atoms that can give a factor below one to any survivor */
            const double lim_n = kappa * dbmax;
            for (int c = 0; c < natom; ++c)
                if (d[c] < lim_n) near[nn++] = c;
            double z = 0.0, pp = 0.0;
            for (int q = 0; q < ns; ++q) {
                const int b = cand[q];
                const double lim = kappa * d[b];
                const double* ir = inv_r + (size_t)b * natom;
                double pb = 1.0;
                for (int k = 0; k < nn && pb != 0.0; ++k) {
                    const int c = near[k];
                    if (c == b || d[c] >= lim) continue;
                    pb *= ssf_s((d[b] - d[c]) * ir[c]);
                }
                z += pb;
                if (b == p) pp = pb;
            }
            out[i] = pp == 0.0 ? 0.0 : pp / z;
        }
        free(d);
        free(cand);
        free(near);
    }
    free(inv_r);
    free(rnn);
    return fail ? -1 : 0;
}
