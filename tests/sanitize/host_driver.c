/* Drives the host-side argument validation of the library's C ABI (basis, grid, weights and
 * option checks, the basis screening radius, status strings) so that a build of the host code
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check it.  No call here reaches a
 * kernel: every context creation either fails validation or, with valid arguments, stops at
 * (or passes) the device selection; a created context is destroyed at once.  Exit status 0 and
 * "host driver ok" on success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "snk.h"

#define EXPECT(call, code, what)                                                            \
    do {                                                                                    \
        const int rc_ = (call);                                                             \
        if (rc_ != (code)) {                                                                \
            fprintf(stderr, "host driver: %s returned %d, expected %d\n", what, rc_, code); \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

int main(void)
{
    double center[6] = {0, 0, 0, 1.0, 0.2, -0.4};
    int32_t l[2] = {1, 0};
    int32_t nprim[2] = {2, 1};
    int32_t prim_off[2] = {0, 2};
    double exps[3] = {2.0, 0.5, 1.1};
    double coefs[3] = {0.6, 0.5, 1.0};
    snk_basis b = {2, center, l, nprim, prim_off, exps, coefs};
    double xyz[12] = {0, 0, 0.5, 0.1, 0.2, 0.3, -1, 0.4, 0, 2, 2, 2};
    double w[4] = {0.1, 0.2, 0.3, 0.4};
    snk_grid g = {4, xyz, NULL};
    snk_opts o;
    snk_opts_default(&o);
    snk_ctx* ctx = NULL;
    double P[16] = {0}, K[16] = {0};

    EXPECT(snk_ctx_create(&b, &g, w, &o, NULL), SNK_E_ARG, "NULL output");
    EXPECT(snk_ctx_create(NULL, &g, w, &o, &ctx), SNK_E_ARG, "NULL basis");
    EXPECT(snk_ctx_create(&b, NULL, w, &o, &ctx), SNK_E_ARG, "NULL grid");
    EXPECT(snk_ctx_create(&b, &g, NULL, &o, &ctx), SNK_E_ARG, "NULL weights");

    l[0] = 3;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "l = 3");
    l[0] = 1;
    nprim[1] = 0;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "nprim = 0");
    nprim[1] = SNK_MAX_NPRIM + 1;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "nprim too large");
    nprim[1] = 1;
    prim_off[1] = -1;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "negative offset");
    prim_off[1] = 2;
    center[4] = NAN;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "NaN centre");
    center[4] = 0.2;
    exps[1] = -0.5;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "negative exponent");
    exps[1] = 0.5;
    coefs[2] = INFINITY;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "infinite coefficient");
    coefs[2] = 1.0;
    b.nshell = 0;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "no shells");
    b.nshell = 2;

    g.npts = -1;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "negative point count");
    g.npts = 4;
    xyz[7] = NAN;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "NaN point");
    xyz[7] = 0.4;
    w[2] = -1e-3;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "negative weight");
    w[2] = 0.3;

    o.precision = (snk_precision)7;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "unknown precision");
    snk_opts_default(&o);
    o.screen = (snk_screen)9;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "unknown screen");
    snk_opts_default(&o);
    o.flags = 0x4u;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "unknown flag");
    snk_opts_default(&o);
    o.batch_points = 300;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "batch_points");
    snk_opts_default(&o);
    o.eps_basis = -1.0;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "negative eps_basis");
    snk_opts_default(&o);
    o.screen = SNK_SCREEN_BOUND;
    o.eps_skip_energy = NAN;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "NaN eps_skip_energy");
    snk_opts_default(&o);
    o.screen = SNK_SCREEN_LEARNED;
    EXPECT(snk_ctx_create(&b, &g, w, &o, &ctx), SNK_E_ARG, "learned screen without a network");
    snk_opts_default(&o);
    EXPECT(sn_k_build(&b, &g, w, NULL, K, &o), SNK_E_ARG, "one-shot NULL P");
    if (!snk_last_error(NULL) || !strlen(snk_last_error(NULL))) {
        fprintf(stderr, "host driver: no error text after a failed call\n");
        return 1;
    }

    /* valid arguments: the device selection succeeds (a GPU is present) or reports a device error */
    const int rc = snk_ctx_create(&b, &g, w, &o, &ctx);
    if (rc != SNK_OK && rc != SNK_E_DEVICE && rc != SNK_E_NOMEM) {
        fprintf(stderr, "host driver: valid create returned %d\n", rc);
        return 1;
    }
    if (rc == SNK_OK) {
        EXPECT(snk_ctx_build(ctx, NULL, K, NULL), SNK_E_ARG, "build with NULL P");
        snk_ctx_destroy(ctx);
    }
    snk_ctx_destroy(NULL);
    (void)P;

    double r = 0.0;
    EXPECT(snk_shell_rcut(1, exps, coefs, 2, 1e-9, &r), SNK_OK, "rcut");
    if (!(r > 0.0 && isfinite(r))) {
        fprintf(stderr, "host driver: rcut %g\n", r);
        return 1;
    }
    EXPECT(snk_shell_rcut(3, exps, coefs, 2, 1e-9, &r), SNK_E_ARG, "rcut l = 3");
    EXPECT(snk_shell_rcut(1, exps, coefs, 0, 1e-9, &r), SNK_E_ARG, "rcut nprim 0");
    EXPECT(snk_shell_rcut(1, exps, coefs, 2, 0.0, &r), SNK_E_ARG, "rcut eps 0");
    EXPECT(snk_shell_rcut(1, exps, coefs, 2, 1e-9, NULL), SNK_E_ARG, "rcut NULL out");
    EXPECT(snk_shell_rcut(0, exps + 2, coefs + 2, 1, 10.0, &r), SNK_OK, "rcut above the peak");
    for (int s = 0; s <= 6; ++s)
        if (!snk_status_string(s)) {
            fprintf(stderr, "host driver: no status string for %d\n", s);
            return 1;
        }
    if (snk_version() != SNK_VERSION) return 1;
    printf("host driver ok\n");
    return 0;
}
