/*
 * Density-fitted Coulomb matrix by the J-engine (Sec. II.B of the sn-K paper): the Fock
 * matrix's Coulomb term in the density-fitting (resolution-of-the-identity) approximation,
 *
 *   v_L  = sum_{lam kap} (L | lam kap) P_{lam kap}                          (Eq. V_df)
 *   d_K  = sum_L (V^-1)_{KL} v_L,   V_{KL} = (K | L)                        (Eq. P_df)
 *   J_{mu nu} = sum_K (mu nu | K) d_K                                       (Eq. J_df)
 *
 * evaluated as in the paper's J-engine: the density of every orbital primitive pair is first
 * contracted with its Hermite expansion coefficients (Eq. Dp), the Hermite Coulomb integrals
 * (Eq. pc, from the auxiliary integrals of Eq. md1 and the Boys function) are digested against
 * those Hermite densities (Eq. cabP-jengine), and for J the auxiliary coefficients are turned
 * into Hermite densities of the auxiliary shells, digested per orbital primitive pair, and
 * transformed back to the Cartesian pair.  The metric V is formed and Cholesky-factorised on
 * the GPU once per context (it depends on the auxiliary basis only); a build costs two
 * triangular solves.  FP64 throughout; every sum is formed in a fixed order (bitwise
 * reproducible); no screening of the three-centre terms.
 *
 * Bases use the snk_basis layout of snk.h (Cartesian shells l <= 2, contraction coefficients
 * for unit-normalised axis-aligned components, the other components scaled the same way as in
 * sn-K).  Auxiliary shells have one primitive each.
 */
#ifndef SNK_DFJ_H
#define SNK_DFJ_H

#include <stdint.h>

#include "snk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snk_dfj snk_dfj;

/*
 * Context for one orbital basis and one auxiliary basis on `device`, its work ordered on
 * `stream` (a hipStream_t, or NULL for the null stream).  Builds the primitive-pair and
 * auxiliary-shell tables, the metric V and its Cholesky factor.  SNK_E_ARG for a NULL
 * pointer, an invalid shell (as for snk_ctx_create), an auxiliary shell with more than one
 * primitive, or an auxiliary basis whose metric is not positive definite (linearly dependent
 * functions); SNK_E_NOMEM / SNK_E_DEVICE for allocation or HIP errors.  The caller owns
 * `*out` and releases it with snk_dfj_destroy.
 */
int snk_dfj_create(const snk_basis* basis, const snk_basis* aux, int device, void* stream, snk_dfj** out);

/*
 * J_out = J[P] (nbf x nbf row-major, both triangles, exactly symmetric).  Optional outputs
 * (NULL to skip): v_out (nauxf) = v of Eq. V_df, d_out (nauxf) = d of Eq. P_df, in the order of
 * the auxiliary functions of the basis given to snk_dfj_create; ej_out (host) = 1/2 tr(P J).
 * flags: SNK_DEVICE_PTRS makes P, J_out, v_out and d_out device pointers and the call
 * asynchronous on the context's stream (returning after ej_out is written when ej_out is not
 * NULL); otherwise they are host pointers and the call returns when they are written.
 * SNK_E_ARG for a NULL ctx, P or J_out or an unknown flag.
 */
int snk_dfj_build(snk_dfj* ctx, const double* P, double* J_out, double* v_out, double* d_out, double* ej_out,
                  uint32_t flags);

/* auxiliary functions (nauxf) of a context; 0 for NULL */
int64_t snk_dfj_naux(const snk_dfj* ctx);
/* error text of the last failed call on ctx */
const char* snk_dfj_last_error(const snk_dfj* ctx);
void snk_dfj_destroy(snk_dfj* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SNK_DFJ_H */
