/*
 * snk_testing.h -- test hooks of the sn-K library (libsnk.so).
 *
 * For the library's own tests: they expose single kernels (the Boys function, the grouped
 * matrix-core product, matrix-core operand layouts) and intermediates of a build, so that
 * each can be checked on its own against host references.  Nothing here is needed to
 * build K; the conventions of snk.h (status codes, ownership, device/host pointers) apply.
 */
#ifndef SNK_TESTING_H
#define SNK_TESTING_H

#include "snk.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Boys function on the device (Eq. boys), as used by the integral kernels:
 * F_m(T[k]) for m = 0..mmax (mmax <= 4) written to F_out[k*(mmax+1) + m].
 * T and F_out are device pointers, n values; ordered on `stream` (hipStream_t or
 * NULL for the default stream).
 */
int snk_boys_device(const double* T, int64_t n, int mmax, double* F_out, void* stream);

/*
 * Test hooks (diagnostics; not needed for building K).
 *
 * snk_debug_gemm_f64: C = A op(B) with the library's grouped FP64 matrix-core product (one
 *   problem) on device pointers: A is M x K row-major (lda), B is K x N row-major (ldb) or,
 *   with bt != 0, N x K row-major; C is M x N row-major (ldc).  tile: output tile of the
 *   kernel, 64 (64 x 64), 128 (128 x 128), 192 (64 rows x 128 columns) or 384 (128 rows x
 *   256 columns), or 0 for the library's own choice.  Synchronous on `stream`.
 * snk_debug_force_tile: every grouped product launched afterwards in the process uses this
 *   output tile (64, 128, 192 or 384 as for snk_debug_gemm_f64), or the library's own choice again
 *   for 0; process-wide, not thread-safe.  SNK_E_ARG for any other value.
 * snk_debug_frow_prefilter: with 0, every build afterwards in the process tests every function
 *   in the F-row restriction of basis screening instead of only those its block bound (the
 *   largest |P| over the basis functions of two centres) leaves; 1 (the default) restores the
 *   prefilter.  Both give the same rows, so the same K bit for bit; process-wide, not
 *   thread-safe.  SNK_E_ARG for any other value.
 * snk_debug_mfma_layout: writes 256 doubles to host memory `out`: element 4*lane + r of
 *   one v_mfma_f64_16x16x4f64 whose inputs encode D[i][j] = 100 j + i (layout check).
 * snk_ctx_point_order: col_to_point[c] (host, nbatches*256 entries) = input index of the
 *   grid point in batch column c, or -1 for a padding slot.
 * snk_ctx_debug_intermediates: for the first batch group only, the collocation matrix
 *   Phi (Eq. collocation), F (Eq. fmat) and G (Eq. gmat), each nbf x ncols row-major in
 *   host memory (ncols = 256 * batches of that group, returned in *ncols_out); elements of
 *   Phi outside their tile's B_t are zero; P is a host pointer.  Pass NULL for any output not
 *   wanted.
 * snk_ctx_npair_index: size of the pair index space, nshell (nshell + 1) / 2 (pair of
 *   shells s >= t at s (s + 1) / 2 + t).
 * snk_ctx_debug_learned: runs the learned screen of the first batch group (context made
 *   with SNK_SCREEN_LEARNED; P a host pointer) and copies to host memory, per batch b of
 *   that group and pair index p, the raw network output yraw[b * npair_index + p] and the
 *   block estimate log2 est[...] (NaN for blocks the bound already skipped), and the
 *   first kept estimate bin thr[b].  *nbatch_out = batches of the group.
 * snk_ctx_debug_kept: runs the first batch group of a context with a density screen (P a
 *   host pointer, host-pointer context) and returns the shell pairs the screen kept for the
 *   A.F step, as int32 triples (batch, A, B) in `out` (A is the shell of larger angular
 *   momentum, or of larger index for equal ones); *n_out = number of triples.  out = NULL
 *   queries the count; cap = triples out holds (SNK_E_ARG when fewer than kept).
 * snk_debug_mfma_bf16: D = A B (16 x 16 row-major host D) through one bf16 matrix-core op,
 *   A and B rounded to bf16: with k32 = 0, A and B are 16 x 16 (16x16x16 op); with k32 != 0,
 *   A is 16 x 32 and B 32 x 16 (16x16x32 op).  Layout check.
 */
int snk_debug_gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                       int64_t ldb, int bt, double* C, int64_t ldc, int tile, void* stream);
int snk_debug_force_tile(int tile);
int snk_debug_frow_prefilter(int on);
int snk_debug_mfma_layout(double* out);
int snk_ctx_point_order(const snk_ctx* ctx, int64_t* col_to_point);
int snk_ctx_debug_intermediates(snk_ctx* ctx, const double* P, double* Phi, double* F, double* G,
                                int64_t* ncols_out);
int64_t snk_ctx_npair_index(const snk_ctx* ctx);
int snk_ctx_debug_learned(snk_ctx* ctx, const double* P, float* yraw, float* est, int32_t* thr,
                          int64_t* nbatch_out);
int snk_ctx_debug_kept(snk_ctx* ctx, const double* P, int32_t* out, int64_t cap, int64_t* n_out);
int snk_debug_mfma_bf16(const float* A, const float* B, float* D, int k32);

#ifdef __cplusplus
}
#endif

#endif /* SNK_TESTING_H */
